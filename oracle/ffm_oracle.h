/*
 * ffm_oracle.h -- FP64 CPU oracle for the Fast Free Memory (FFM) method.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product library
 * never calls it, and the two share no code.
 *
 * Everything is plain, slow and direct: FP64 real arithmetic, C99 complex
 * (complex128) accumulation, OpenMP only over independent boxes or rows.
 *
 * Paper: Aussal & Bakry, "The Fast and Free Memory Method for the efficient
 * computation of convolution kernels" (arXiv:1909.05600).
 *   - operator v_i = sum_j w_j G(x_i, y_j) u_j         : Sec. 1, eqs. (convolution_discrete), (convolution_matrix)
 *   - root cubes, d_l = d_0 / 2^l                       : Sec. 2.2.1
 *   - admissibility and Lagrange interpolation          : Sec. 2.2.2
 *   - Gegenbauer plane-wave form for Helmholtz          : Sec. 2.2.3, eqs. (gegenbauerIntegral..gegenbauerQuadrature)
 *   - stopping criterion and dense remainder            : Sec. 2.2.4
 *   - descent-only traversal, reuse per translation     : Sec. 3.1-3.2 (proof of Prop. 1)
 *   - kernels: Laplace (laplaceGreenKernel), Helmholtz (helmholtzKernel)
 *
 * Complex arrays are interleaved (re, im) doubles.  Coordinates are n x 3
 * row-major doubles.  All indices are 64-bit.
 */
#ifndef FFM_ORACLE_H
#define FFM_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define ORC_LAPLACE 0
#define ORC_HELMHOLTZ 1
/* The normal derivative at the target, dG/dn_x (x, y) = n_x . grad_x G(x - y): the kernel of the adjoint
 * double-layer operator (Sec. 4.2.1, eq. doubleLayer), for each base kernel; plans need target normals. */
#define ORC_LAPLACE_DN 2
#define ORC_HELMHOLTZ_DN 3
/* The normal derivative at the source, dG/dn_y (x, y) = n_y . grad_y G(x - y): the kernel of the double-layer
 * operator (Sec. 4.2.1, eq. doubleLayer), for each base kernel; plans need source normals. */
#define ORC_LAPLACE_DL 4
#define ORC_HELMHOLTZ_DL 5
/* The gradient at the target, grad_x G(x - y) (three components per target; the vector kernels of the
 * integral operators of Sec. 4.2.2), for each base kernel; plans write v as n_x x 3 complex values. */
#define ORC_LAPLACE_GRAD 6
#define ORC_HELMHOLTZ_GRAD 7

/* ---- plain definition ---------------------------------------------------- */
/* out[a] = sum_{j : |x_rows[a] - y_j| > 0} G(|x_rows[a] - y_j|) * wu[j]  (complex128 out) */
void orc_dense_rows(const double *X, const double *Y, int64_t ny, const double *wu,
                    int kernel, double k, const int64_t *rows, int64_t nrows, double *out);

/* out[a] = sum_{j : |x - y_j| > 0} n_x . grad_x G(x - y_j) wu[j] at x = x_rows[a] with normal NX[rows[a]];
 * kernel ORC_LAPLACE or ORC_HELMHOLTZ (the base kernel) */
void orc_dense_rows_dn(const double *X, const double *Y, int64_t ny, const double *wu, int kernel, double k,
                       const double *NX, const int64_t *rows, int64_t nrows, double *out);
/* out[a] = sum_{j : |x - y_j| > 0} n_j . grad_y G(x - y_j) wu[j] at x = x_rows[a] with source normals NY (ny x 3);
 * kernel ORC_LAPLACE or ORC_HELMHOLTZ (the base kernel) */
/* out[a][c] = sum_{j : |x - y_j| > 0} d/dx_c G(x - y_j) wu[j] at x = x_rows[a], c = 0, 1, 2 (out: nrows x 3
 * complex); kernel ORC_LAPLACE or ORC_HELMHOLTZ (the base kernel) */
void orc_dense_rows_grad(const double *X, const double *Y, int64_t ny, const double *wu, int kernel, double k,
                         const int64_t *rows, int64_t nrows, double *out);
void orc_dense_rows_dl(const double *X, const double *Y, int64_t ny, const double *wu, int kernel, double k,
                       const double *NY, const int64_t *rows, int64_t nrows, double *out);

/* ---- building blocks, exported so the tests can pin them ----------------- */
void orc_gauss_legendre(int n, double *x, double *w);
void orc_legendre_p(int L, double t, double *P);                 /* P_0..P_L at t            */
void orc_sph_hankel1(int L, double z, double *h);                 /* h_0..h_L (complex) at z>0 */
void orc_cheb_nodes(int r1, double *t);                           /* first-kind nodes         */
void orc_lagrange_basis(int r1, double t, double *ell);            /* l_1..l_r1 at t           */
void orc_lagrange_basis_deriv(int r1, double t, double *dell);     /* l_1'..l_r1' at t         */
int  orc_gegenbauer_rank(double k, double d_l, double eps);
/* quadrature of a Gegenbauer level: s (nq x 3), w (nq); returns nq = 2L(L+1) */
int64_t orc_sphere_quadrature(int L, double *s, double *w);
/* transfer diagonal D(q) = (ik/4pi) w_q T_{L,r0}(s_q) for one translation r0 (complex out, nq) */
void orc_gegenbauer_diag(int L, double k, const double r0[3], double *D);

/* Grid form of the plane-wave transforms of one box (reading R16-R18; the fast evaluation of the
 * transforms asked for in the remark closing Sec. 2.2.3).  Grid: p nodes per axis at spacing h,
 * node a at (a - (p-1)/2) h from the box centre; kernel phi(t) = exp(beta (sqrt(1 - (2t/w)^2) - 1)),
 * |t| < w/2 (t in node units); directions: the level's quadrature (orc_sphere_quadrature(L)).
 *   forward:  ut(q)  = Phi(q)^-1 sum_abc e^{-ik s_q.x_abc} sum_j u_j phi phi phi((x_abc - y_j)/h)
 *   backward: v_i   += sum_abc phi phi phi((x_abc - x_i)/h) Phi(q)^-1 sum_q e^{ik s_q.x_abc} vt(q)
 * with Phi(q) = prod_d phihat(k s_qd h), phihat(xi) = integral of phi(t) e^{-i xi t} dt.
 * Points are box-relative (n x 3); u, ut, vt, v complex (interleaved); v is accumulated. */
void orc_grid_forward(int p, int w, double beta, double h, double k, int L, const double *y, const double *u,
                      int64_t n, double *ut);
void orc_grid_backward(int p, int w, double beta, double h, double k, int L, const double *vt, const double *x,
                       int64_t n, double *v);
/* phihat(xi) of the kernel above (Gauss-Legendre after t = (w/2) sin(theta)) */
double orc_es_hat(int w, double beta, double xi);

/* Adaptive cross approximation with complete pivoting of an r x r complex matrix T (row-major, interleaved):
 * T ~ A B^T, A and B r x rank column-major complex (caller provides r x r each); returns the rank, the
 * fewest greedy cross terms with |T - A B^T|_F <= tol |T|_F (Sec. 2.2.2, eq. ffmACAmatvec; reading R21). */
int orc_aca(int r, const double *T, double tol, double *A, double *B);

/* ---- plan ----------------------------------------------------------------- */
typedef struct orc_plan orc_plan;

#define ORC_MAX_LEVELS 21

typedef struct {
    int32_t n_leaf;       /* occupancy threshold of the stopping rule (default 64) */
    double  kappa;        /* Gegenbauer iff k*d_l >= kappa (default pi)             */
    int32_t r1_override;  /* > 0: Chebyshev nodes per axis at every Lagrange level */
    int32_t max_level;    /* depth cap (default 20)                                 */
    /* Grid form of the plane-wave transforms of Gegenbauer level l (reading R16-R18): grid_p[l] > 0
     * nodes per axis, kernel width grid_w[l] nodes, shape grid_beta[l]; 0 = direct sums. */
    int32_t grid_p[ORC_MAX_LEVELS];
    int32_t grid_w[ORC_MAX_LEVELS];
    double  grid_beta[ORC_MAX_LEVELS];
    /* ACA of the Lagrange transfer matrices (Sec. 2.2.2, eq. ffmACAmatvec) at the levels with aca[l] != 0,
     * relative tolerance aca_tol (reading R21); 0 = plain transfer matrices. */
    double  aca_tol;
    int32_t aca[ORC_MAX_LEVELS];
    /* ORC_*_DN kernels: unit normals at the targets, n_x x 3, user order (copied at plan creation) */
    const double *target_normals;
    /* per-pair leaf rule (reading R22): near pairs whose boxes both hold <= n_leaf points are summed densely at
     * their level instead of refined */
    int32_t adaptive;
    /* ORC_*_DL kernels: unit normals at the sources, n_y x 3, user order (copied at plan creation) */
    const double *source_normals;
} orc_options;

orc_plan *orc_plan_create(const double *X, int64_t nx, const double *Y, int64_t ny,
                          int kernel, double k, double eps, const orc_options *opt);
void orc_plan_free(orc_plan *p);

/* apply: v (complex, user target order) = FFM(wu (complex, user source order)); gradient plans write n_x x 3
 * values, v[3 i + c] the c-th component at target i.
 * stride > 1 evaluates, in every per-point loop (transforms, near-field targets),
 * only the points whose sorted index is a multiple of stride, keeping every box,
 * table and transfer: a bounded timing sample whose result is not the product. */
void orc_apply(orc_plan *p, const double *wu, double *v, int64_t stride);

/* ---- queries for bit-exact comparison ------------------------------------- */
int     orc_num_threads(void);                                     /* OpenMP threads used      */
int     orc_leaf(const orc_plan *p);
double  orc_d0(const orc_plan *p);
void    orc_corner(const orc_plan *p, int set, double *c3);        /* set 0 = X (targets), 1 = Y */
int64_t orc_npoints(const orc_plan *p, int set);
void    orc_keys(const orc_plan *p, int set, uint64_t *keys);       /* sorted keys               */
void    orc_perm(const orc_plan *p, int set, int64_t *perm);        /* sorted pos -> user index  */
int64_t orc_nbox(const orc_plan *p, int set, int l);
void    orc_box_start(const orc_plan *p, int set, int l, int64_t *start);  /* nbox+1 entries */
void    orc_box_ijk(const orc_plan *p, int set, int l, int32_t *ijk);      /* nbox x 3       */
void    orc_box_centre(const orc_plan *p, int set, int l, double *c);      /* nbox x 3       */
int64_t orc_nfar(const orc_plan *p, int l);
void    orc_far(const orc_plan *p, int l, int64_t *t, int64_t *s, int32_t *off); /* off: nfar x 3 */
int64_t orc_nnear(const orc_plan *p, int l);                        /* near_l (valid l <= leaf) */
void    orc_near(const orc_plan *p, int l, int64_t *t, int64_t *s);
int64_t orc_nearly(const orc_plan *p, int l);                       /* pairs the per-pair rule stopped at l */
void    orc_early(const orc_plan *p, int l, int64_t *t, int64_t *s);
int     orc_level_method(const orc_plan *p, int l);                 /* 0 none, 1 Lagrange, 2 Gegenbauer */
int     orc_level_order(const orc_plan *p, int l);                  /* r1 or L                   */
/* ACA ranks of the transfer matrices of Lagrange level l at tolerance tol: one per translation class, with
 * its integer offset (off: n x 3); returns the number of classes n (caller sizes off and ranks >= 316). */
int     orc_aca_ranks(const orc_plan *p, int l, double tol, int32_t *off, int32_t *ranks);

#ifdef __cplusplus
}
#endif
#endif
