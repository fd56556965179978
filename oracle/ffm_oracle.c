/*
 * ffm_oracle.c -- FP64 CPU oracle for the Fast Free Memory method.
 *
 * TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU baseline
 * leg of the benchmark load this file's library.  It shares no code with the
 * GPU library.  Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off (the
 * geometry steps must round every operation separately).
 *
 * The FFM approximates the discrete convolution of Sec. 1 (eqs.
 * convolution_discrete / convolution_matrix) by a descent over two octrees
 * with cubic roots of the same edge (Sec. 2.1, 2.2.1).  At every level the
 * admissible ("far") box pairs are compressed either by Chebyshev/Lagrange
 * interpolation (Sec. 2.2.2) or, for oscillatory Helmholtz levels, by the
 * Gegenbauer plane-wave form (Sec. 2.2.3); the other pairs are split into
 * their children.  The descent stops by the rule of Sec. 2.2.4 and the
 * remaining pairs are summed densely.
 *
 * Readings where the paper is silent or ambiguous (each also listed in the
 * design notes):
 *   R1  each root cube is centred on its set's bounding box; the cube edge d_0
 *       is the largest bounding-box edge over both sets (d_0 = 1 if zero).
 *   R2  a pair is admissible iff the max-norm distance of the box centres is
 *       >= 2 d_l.  This reproduces the 2-D counts of the proof of Prop. 1
 *       (27 interactions of an interior box, 40 distinct translations).
 *   R3  the root pair is near; classification starts at level 1.
 *   R4  stop at the first level l >= 1 whose near list is empty, or whose
 *       average occupancy (N_X+N_Y)/(nb_X+nb_Y) is <= n_leaf (integer test),
 *       or at the depth cap.
 *   R5  Chebyshev nodes of the first kind, r1 = ceil(ln(1/eps)/ln(3+sqrt 8))
 *       per axis (+ ceil(k d_l / 2) at Helmholtz Lagrange levels).
 *   R6  Helmholtz levels use the Gegenbauer form iff k d_l >= kappa (pi).
 *   R7  L = floor(k sqrt(3) d_l - ln eps) with the natural log, L >= 1.
 *   R8  the Gegenbauer series starts at p = 0.
 *   R9  box-centred coordinates and no extra phase factor:
 *       G ~ sum_q e^{ik s_q.(x-x0)} D(q) e^{-ik s_q.(y-y0)},
 *       D(q) = (ik/4pi) w_q T_{L,r0}(s_q), r0 = x0 - y0.
 *   R10 quadrature: (L+1) Gauss-Legendre nodes in cos(theta) times 2L
 *       equispaced phi = pi n / L, weight w_m pi / L  (n_Q = 2L(L+1)).
 *   R11 coincident points (r == 0) contribute nothing.
 *   R12 Morton keys: 21 bits per axis, x in the highest bit of each triple.
 *   R16-R18 grid form of the transforms (optional per level, parameters given
 *       by the caller): exponential-of-semicircle kernel of width w nodes and
 *       shape beta on a p^3 grid of spacing h = d_l / (p - 1 - w) about the box
 *       centre, the kernel's Fourier transform divided out per direction.
 */
#include "ffm_oracle.h"

#include <complex.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define BITS 21
#define QMAX ((int64_t)1 << BITS)
#define ORC_PI 3.14159265358979323846

/* =========================================================================
 * Kernels (Sec. 4.1 eq. laplaceGreenKernel; Sec. 2.2.3 eq. helmholtzKernel)
 * ========================================================================= */
static double complex green(int kernel, double k, double r)
{
    if (kernel == ORC_LAPLACE) return 1.0 / (4.0 * ORC_PI * r);
    return cexp(I * (k * r)) / (4.0 * ORC_PI * r);
}

/* Normal derivative at the target, n . grad_x G(x - y) with d = x - y (the adjoint double-layer kernel of
 * Sec. 4.2.1, eq. doubleLayer): grad_x G = d G'(r) / r, G'(r) = -1 / (4 pi r^2) (Laplace) or
 * (ikr - 1) e^{ikr} / (4 pi r^2) (Helmholtz). */
static double complex green_dn(int kernel, double k, const double d[3], const double n[3])
{
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double nd = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
    const double r3 = 4.0 * ORC_PI * r * r * r;
    if (kernel == ORC_LAPLACE) return -nd / r3;
    return nd * (I * (k * r) - 1.0) * cexp(I * (k * r)) / r3;
}

/* Normal derivative at the source, n . grad_y G(x - y) with d = x - y (the double-layer kernel of Sec. 4.2.1,
 * eq. doubleLayer): grad_y G(x - y) = -grad_x G(x - y), so it is green_dn with the source normal and the
 * opposite sign. */
static double complex green_dl(int kernel, double k, const double d[3], const double n[3])
{
    return -green_dn(kernel, k, d, n);
}

/* Timing samples (orc_apply with stride > 1) keep the points whose sorted index is a multiple of the stride:
 * the first such index at or after i. */
static int64_t first_sample(int64_t i, int64_t stride) { return (i + stride - 1) / stride * stride; }

static double complex cload(const double *a, int64_t i) { return a[2 * i] + I * a[2 * i + 1]; }

/* The plain definition (Sec. 1, eq. convolution_discrete) on sampled rows. */
void orc_dense_rows(const double *X, const double *Y, int64_t ny, const double *wu,
                    int kernel, double k, const int64_t *rows, int64_t nrows, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t a = 0; a < nrows; ++a) {
        const double *x = X + 3 * rows[a];
        double complex acc = 0.0;
        for (int64_t j = 0; j < ny; ++j) {
            double dx = x[0] - Y[3 * j], dy = x[1] - Y[3 * j + 1], dz = x[2] - Y[3 * j + 2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;                       /* R11 */
            acc += green(kernel, k, sqrt(r2)) * cload(wu, j);
        }
        out[2 * a] = creal(acc);
        out[2 * a + 1] = cimag(acc);
    }
}

/* =========================================================================
 * Special functions and quadratures
 * ========================================================================= */

/* Legendre polynomials by Bonnet's recurrence. */
void orc_legendre_p(int L, double t, double *P)
{
    P[0] = 1.0;
    if (L >= 1) P[1] = t;
    for (int p = 1; p < L; ++p) P[p + 1] = ((2.0 * p + 1.0) * t * P[p] - p * P[p - 1]) / (p + 1.0);
}

/* Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_n. */
void orc_dense_rows_dn(const double *X, const double *Y, int64_t ny, const double *wu, int kernel, double k,
                       const double *NX, const int64_t *rows, int64_t nrows, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < nrows; ++a) {
        const double *x = X + 3 * rows[a];
        const double *n = NX + 3 * rows[a];
        double complex acc = 0.0;
        for (int64_t j = 0; j < ny; ++j) {
            double d[3] = {x[0] - Y[3 * j], x[1] - Y[3 * j + 1], x[2] - Y[3 * j + 2]};
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] == 0.0) continue;   /* R11 */
            acc += green_dn(kernel, k, d, n) * cload(wu, j);
        }
        out[2 * a] = creal(acc);
        out[2 * a + 1] = cimag(acc);
    }
}

void orc_dense_rows_grad(const double *X, const double *Y, int64_t ny, const double *wu, int kernel, double k,
                         const int64_t *rows, int64_t nrows, double *out)
{
    static const double axis[3][3] = {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}};
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < nrows; ++a) {
        const double *x = X + 3 * rows[a];
        double complex acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < ny; ++j) {
            double d[3] = {x[0] - Y[3 * j], x[1] - Y[3 * j + 1], x[2] - Y[3 * j + 2]};
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] == 0.0) continue;   /* R11 */
            for (int c = 0; c < 3; ++c) acc[c] += green_dn(kernel, k, d, axis[c]) * cload(wu, j);
        }
        for (int c = 0; c < 3; ++c) {
            out[2 * (3 * a + c)] = creal(acc[c]);
            out[2 * (3 * a + c) + 1] = cimag(acc[c]);
        }
    }
}

void orc_dense_rows_dl(const double *X, const double *Y, int64_t ny, const double *wu, int kernel, double k,
                       const double *NY, const int64_t *rows, int64_t nrows, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < nrows; ++a) {
        const double *x = X + 3 * rows[a];
        double complex acc = 0.0;
        for (int64_t j = 0; j < ny; ++j) {
            double d[3] = {x[0] - Y[3 * j], x[1] - Y[3 * j + 1], x[2] - Y[3 * j + 2]};
            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] == 0.0) continue;   /* R11 */
            acc += green_dl(kernel, k, d, NY + 3 * j) * cload(wu, j);
        }
        out[2 * a] = creal(acc);
        out[2 * a + 1] = cimag(acc);
    }
}

void orc_gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5));
        double pn = 0.0, pm = 0.0, dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            pm = 1.0;
            pn = z;
            for (int j = 1; j < n; ++j) {
                double nx = ((2.0 * j + 1.0) * z * pn - j * pm) / (j + 1.0);
                pm = pn;
                pn = nx;
            }
            dp = n * (z * pn - pm) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* re-evaluate the derivative at the converged node for the weight */
        pm = 1.0;
        pn = z;
        for (int j = 1; j < n; ++j) {
            double nx = ((2.0 * j + 1.0) * z * pn - j * pm) / (j + 1.0);
            pm = pn;
            pn = nx;
        }
        dp = n * (z * pn - pm) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Spherical Hankel functions of the first kind h_p = j_p + i y_p, p = 0..L, by upward
 * recurrence from h_0 = -i e^{iz}/z and h_1 = -e^{iz}(z + i)/z^2. */
void orc_sph_hankel1(int L, double z, double *h)
{
    double complex e = cexp(I * z);
    double complex hm = -I * e / z;
    h[0] = creal(hm);
    h[1] = cimag(hm);
    if (L < 1) return;
    double complex hp = -e * (z + I) / (z * z);
    h[2] = creal(hp);
    h[3] = cimag(hp);
    for (int p = 1; p < L; ++p) {
        double complex hn = (2.0 * p + 1.0) / z * hp - hm;
        hm = hp;
        hp = hn;
        h[2 * (p + 1)] = creal(hp);
        h[2 * (p + 1) + 1] = cimag(hp);
    }
}

/* Chebyshev nodes of the first kind, t_a = cos((2a-1) pi / (2 r1)), a = 1..r1 (R5). */
void orc_cheb_nodes(int r1, double *t)
{
    for (int a = 1; a <= r1; ++a) t[a - 1] = cos((2.0 * a - 1.0) * ORC_PI / (2.0 * r1));
}

/* One-dimensional Lagrange polynomials on the Chebyshev nodes evaluated at t. */
void orc_lagrange_basis(int r1, double t, double *ell)
{
    double nodes[64];
    orc_cheb_nodes(r1, nodes);
    for (int a = 0; a < r1; ++a) {
        double v = 1.0;
        for (int b = 0; b < r1; ++b)
            if (b != a) v *= (t - nodes[b]) / (nodes[a] - nodes[b]);
        ell[a] = v;
    }
}

/* Derivatives of the one-dimensional Lagrange polynomials at t:
 * l_a'(t) = sum_{m != a} prod_{b != a, m} (t - t_b) / prod_{b != a} (t_a - t_b). */
void orc_lagrange_basis_deriv(int r1, double t, double *dell)
{
    double nodes[64];
    orc_cheb_nodes(r1, nodes);
    for (int a = 0; a < r1; ++a) {
        double den = 1.0, sum = 0.0;
        for (int b = 0; b < r1; ++b)
            if (b != a) den *= nodes[a] - nodes[b];
        for (int m = 0; m < r1; ++m) {
            if (m == a) continue;
            double pr = 1.0;
            for (int b = 0; b < r1; ++b)
                if (b != a && b != m) pr *= t - nodes[b];
            sum += pr;
        }
        dell[a] = sum / den;
    }
}

/* Truncation rank of the Gegenbauer series, eq. (gegenbauerRank) with the natural log (R7). */
int orc_gegenbauer_rank(double k, double d_l, double eps)
{
    int L = (int)floor(k * sqrt(3.0) * d_l - log(eps));
    return L < 1 ? 1 : L;
}

/* Spherical quadrature of Sec. 3.3 (n_Q = 2L(L+1)), laid out theta-major (R10). */
int64_t orc_sphere_quadrature(int L, double *s, double *w)
{
    int nth = L + 1, nph = 2 * L;
    double *xm = malloc(sizeof(double) * nth), *wm = malloc(sizeof(double) * nth);
    orc_gauss_legendre(nth, xm, wm);
    for (int m = 0; m < nth; ++m) {
        double ct = xm[m], st = sqrt(1.0 - ct * ct);
        for (int n = 0; n < nph; ++n) {
            double ph = ORC_PI * n / L;
            int64_t q = (int64_t)m * nph + n;
            s[3 * q] = st * cos(ph);
            s[3 * q + 1] = st * sin(ph);
            s[3 * q + 2] = ct;
            w[q] = wm[m] * ORC_PI / L;
        }
    }
    free(xm);
    free(wm);
    return (int64_t)nth * nph;
}

/* D(q) = (ik/4pi) w_q T_{L,r0}(s_q), with the Gegenbauer series of eq. (gegenbauerSerie)
 * summed from p = 0 (R8):  T_{L,r0}(s) = sum_p (2p+1) i^p h_p(k|r0|) P_p(s . r0/|r0|) / (4 pi). */
static void gegenbauer_diag_q(int L, double k, const double r0[3], const double *s, const double *w,
                              int64_t nq, double complex *D)
{
    double rn = sqrt(r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2]);
    double *h = malloc(sizeof(double) * 2 * (L + 1));
    double *P = malloc(sizeof(double) * (L + 1));
    double complex *c = malloc(sizeof(double complex) * (L + 1));
    orc_sph_hankel1(L, k * rn, h);
    double complex ip = 1.0;
    for (int p = 0; p <= L; ++p) {
        c[p] = (2.0 * p + 1.0) * ip * (h[2 * p] + I * h[2 * p + 1]) / (4.0 * ORC_PI);
        ip *= I;
    }
    for (int64_t q = 0; q < nq; ++q) {
        double t = (s[3 * q] * r0[0] + s[3 * q + 1] * r0[1] + s[3 * q + 2] * r0[2]) / rn;
        orc_legendre_p(L, t, P);
        double complex T = 0.0;
        for (int p = 0; p <= L; ++p) T += c[p] * P[p];
        D[q] = (I * k / (4.0 * ORC_PI)) * w[q] * T;
    }
    free(h);
    free(P);
    free(c);
}

void orc_gegenbauer_diag(int L, double k, const double r0[3], double *D)
{
    int64_t nq = 2 * (int64_t)L * (L + 1);
    double *s = malloc(sizeof(double) * 3 * nq), *w = malloc(sizeof(double) * nq);
    orc_sphere_quadrature(L, s, w);
    gegenbauer_diag_q(L, k, r0, s, w, nq, (double complex *)D);
    free(s);
    free(w);
}

/* =========================================================================
 * Grid form of the plane-wave transforms (readings R16-R18).  The remark closing
 * Sec. 2.2.3 asks for the transforms of a Gegenbauer level to be evaluated fast
 * rather than as full sums.  The reading taken: spread the points onto a uniform
 * grid about the box centre with a smooth kernel phi, sum the grid values against
 * the plane waves (separably: over z per ring of directions, then over the plane per
 * direction), and divide by the kernel's Fourier transform.  By Poisson summation,
 * sum_a phi((x_a - y)/h) e^{-i om x_a} = e^{-i om y} phihat(om h) + aliased terms,
 * so each axis is exact up to the aliased terms.
 * ========================================================================= */
static double es_phi(double t, int w, double beta)
{
    double x = 2.0 * t / w, s = 1.0 - x * x;
    return s > 0.0 ? exp(beta * (sqrt(s) - 1.0)) : 0.0;
}

/* integral over |t| < w/2 of phi(t) cos(xi t) dt, with t = (w/2) sin(theta): the integrand
 * (w/2) cos(theta) exp(beta (cos(theta) - 1)) cos(xi t) is smooth on |theta| <= pi/2 */
static double es_hat_nodes(int w, double beta, double xi, const double *gx, const double *gw, int n)
{
    double a = 0.0;
    for (int j = 0; j < n; ++j) {
        double th = 0.5 * ORC_PI * gx[j];
        double t = 0.5 * w * sin(th);
        a += gw[j] * (0.5 * ORC_PI) * (0.5 * w) * cos(th) * exp(beta * (cos(th) - 1.0)) * cos(xi * t);
    }
    return a;
}

#define ES_HAT_NODES 96

double orc_es_hat(int w, double beta, double xi)
{
    double gx[ES_HAT_NODES], gw[ES_HAT_NODES];
    orc_gauss_legendre(ES_HAT_NODES, gx, gw);
    return es_hat_nodes(w, beta, xi, gx, gw, ES_HAT_NODES);
}

typedef struct {
    int p, w, L;
    double beta, h, k;
    int64_t nq;
    double *s, *wq;    /* the level's quadrature directions and weights */
    double *Phi;       /* Phi(q) = prod_d phihat(k s_qd h) */
} gridlev_t;

static void gridlev_init(gridlev_t *g, int p, int w, double beta, double h, double k, int L)
{
    g->p = p;
    g->w = w;
    g->L = L;
    g->beta = beta;
    g->h = h;
    g->k = k;
    g->nq = 2 * (int64_t)L * (L + 1);
    g->s = malloc(sizeof(double) * 3 * g->nq);
    g->wq = malloc(sizeof(double) * g->nq);
    g->Phi = malloc(sizeof(double) * g->nq);
    orc_sphere_quadrature(L, g->s, g->wq);
    double gx[ES_HAT_NODES], gw[ES_HAT_NODES];
    orc_gauss_legendre(ES_HAT_NODES, gx, gw);
    for (int64_t q = 0; q < g->nq; ++q) {
        double f = 1.0;
        for (int d = 0; d < 3; ++d) f *= es_hat_nodes(w, beta, k * g->s[3 * q + d] * h, gx, gw, ES_HAT_NODES);
        g->Phi[q] = f;
    }
}

static void gridlev_free(gridlev_t *g)
{
    free(g->s);
    free(g->wq);
    free(g->Phi);
}

/* The w nodes whose kernel support holds grid coordinate t (node units): a with -w/2 < a - t <= w/2,
 * kept inside the grid; their weights phi(a - t). */
static int spread_nodes(double t, int p, int w, double beta, double *wt)
{
    int lo = (int)floor(t - 0.5 * w) + 1;
    if (lo > p - w) lo = p - w;
    if (lo < 0) lo = 0;
    for (int i = 0; i < w; ++i) wt[i] = es_phi(lo + i - t, w, beta);
    return lo;
}

static void grid_fwd(const gridlev_t *g, const double *y, const double complex *u, int64_t n, double complex *ut)
{
    const int p = g->p, w = g->w, nth = g->L + 1, nph = 2 * g->L;
    const double half = 0.5 * (p - 1), h = g->h, k = g->k;
    double complex *G = calloc((size_t)p * p * p, sizeof(double complex));
    double wx[16], wy[16], wz[16];
    /* spreading: G[a][b][c] = sum_j u_j phi phi phi */
    for (int64_t j = 0; j < n; ++j) {
        int a0 = spread_nodes(y[3 * j] / h + half, p, w, g->beta, wx);
        int b0 = spread_nodes(y[3 * j + 1] / h + half, p, w, g->beta, wy);
        int c0 = spread_nodes(y[3 * j + 2] / h + half, p, w, g->beta, wz);
        for (int ia = 0; ia < w; ++ia)
            for (int ib = 0; ib < w; ++ib)
                for (int ic = 0; ic < w; ++ic)
                    G[((size_t)(a0 + ia) * p + (b0 + ib)) * p + (c0 + ic)] += u[j] * wx[ia] * wy[ib] * wz[ic];
    }
    double complex *H = malloc(sizeof(double complex) * (size_t)p * p);
    double complex *ex = malloc(sizeof(double complex) * p), *ey = malloc(sizeof(double complex) * p);
    double complex *ez = malloc(sizeof(double complex) * p);
    for (int m = 0; m < nth; ++m) {
        /* sums over z for ring m (all its directions share cos(theta)) */
        const double ct = g->s[3 * ((int64_t)m * nph) + 2];
        for (int c = 0; c < p; ++c) ez[c] = cexp(-I * k * ct * ((c - half) * h));
        for (int a = 0; a < p; ++a)
            for (int b = 0; b < p; ++b) {
                double complex acc = 0.0;
                for (int c = 0; c < p; ++c) acc += ez[c] * G[((size_t)a * p + b) * p + c];
                H[(size_t)a * p + b] = acc;
            }
        /* sums over the plane for every direction of the ring */
        for (int nn = 0; nn < nph; ++nn) {
            const int64_t q = (int64_t)m * nph + nn;
            for (int a = 0; a < p; ++a) {
                ex[a] = cexp(-I * k * g->s[3 * q] * ((a - half) * h));
                ey[a] = cexp(-I * k * g->s[3 * q + 1] * ((a - half) * h));
            }
            double complex acc = 0.0;
            for (int a = 0; a < p; ++a) {
                double complex row = 0.0;
                for (int b = 0; b < p; ++b) row += ey[b] * H[(size_t)a * p + b];
                acc += ex[a] * row;
            }
            ut[q] = acc / g->Phi[q];
        }
    }
    free(G);
    free(H);
    free(ex);
    free(ey);
    free(ez);
}

static void grid_bwd(const gridlev_t *g, const double complex *vt, const double *x, int64_t n, double complex *v)
{
    const int p = g->p, w = g->w, nth = g->L + 1, nph = 2 * g->L;
    const double half = 0.5 * (p - 1), h = g->h, k = g->k;
    double complex *F = calloc((size_t)p * p * p, sizeof(double complex));
    double complex *K = malloc(sizeof(double complex) * (size_t)p * p);
    double complex *ex = malloc(sizeof(double complex) * p), *ey = malloc(sizeof(double complex) * p);
    double complex *ez = malloc(sizeof(double complex) * p);
    for (int m = 0; m < nth; ++m) {
        /* K[a][b] = sum over the ring's directions of e^{ik (s_x x_a + s_y y_b)} vt(q) / Phi(q) */
        for (size_t i = 0; i < (size_t)p * p; ++i) K[i] = 0.0;
        for (int nn = 0; nn < nph; ++nn) {
            const int64_t q = (int64_t)m * nph + nn;
            for (int a = 0; a < p; ++a) {
                ex[a] = cexp(I * k * g->s[3 * q] * ((a - half) * h));
                ey[a] = cexp(I * k * g->s[3 * q + 1] * ((a - half) * h));
            }
            const double complex f = vt[q] / g->Phi[q];
            for (int a = 0; a < p; ++a)
                for (int b = 0; b < p; ++b) K[(size_t)a * p + b] += ex[a] * ey[b] * f;
        }
        /* F[a][b][c] += e^{ik cos(theta) z_c} K[a][b] */
        const double ct = g->s[3 * ((int64_t)m * nph) + 2];
        for (int c = 0; c < p; ++c) ez[c] = cexp(I * k * ct * ((c - half) * h));
        for (int a = 0; a < p; ++a)
            for (int b = 0; b < p; ++b)
                for (int c = 0; c < p; ++c) F[((size_t)a * p + b) * p + c] += ez[c] * K[(size_t)a * p + b];
    }
    /* interpolation at the targets with the same kernel */
    double wx[16], wy[16], wz[16];
    for (int64_t i = 0; i < n; ++i) {
        int a0 = spread_nodes(x[3 * i] / h + half, p, w, g->beta, wx);
        int b0 = spread_nodes(x[3 * i + 1] / h + half, p, w, g->beta, wy);
        int c0 = spread_nodes(x[3 * i + 2] / h + half, p, w, g->beta, wz);
        double complex acc = 0.0;
        for (int ia = 0; ia < w; ++ia)
            for (int ib = 0; ib < w; ++ib)
                for (int ic = 0; ic < w; ++ic)
                    acc += wx[ia] * wy[ib] * wz[ic] * F[((size_t)(a0 + ia) * p + (b0 + ib)) * p + (c0 + ic)];
        v[i] += acc;
    }
    free(F);
    free(K);
    free(ex);
    free(ey);
    free(ez);
}

void orc_grid_forward(int p, int w, double beta, double h, double k, int L, const double *y, const double *u,
                      int64_t n, double *ut)
{
    gridlev_t g;
    gridlev_init(&g, p, w, beta, h, k, L);
    grid_fwd(&g, y, (const double complex *)u, n, (double complex *)ut);
    gridlev_free(&g);
}

void orc_grid_backward(int p, int w, double beta, double h, double k, int L, const double *vt, const double *x,
                       int64_t n, double *v)
{
    gridlev_t g;
    gridlev_init(&g, p, w, beta, h, k, L);
    grid_bwd(&g, (const double complex *)vt, x, n, (double complex *)v);
    gridlev_free(&g);
}

/* =========================================================================
 * Adaptive cross approximation of a transfer matrix (Sec. 2.2.2, eq. ffmACAmatvec):
 * T ~ A B^T with A, B of r_T columns, by Bebendorf's cross approximation with
 * complete pivoting (reading R21).  Step k takes the largest entry (i_k, j_k) of the
 * residual R_k = T - sum_{l<k} a_l b_l^T and sets a_k = R_k(:, j_k),
 * b_k = R_k(i_k, :) / R_k(i_k, j_k); it stops as soon as |R_k|_F <= tol |T|_F, so the
 * factors meet the tolerance exactly.  The pivot is the first entry in row-major
 * order whose squared modulus is within a relative 2e-9 of the largest, so that
 * entries equal up to rounding (the tensor grid is symmetric) pick the same pivot.
 * ========================================================================= */
typedef double complex (*entry_fn)(const void *ctx, int i, int j);

/* A, B: r x r column-major (column l at A + l r); returns the rank. */
static int aca_factor(int r, entry_fn entry, const void *ctx, double tol, double complex *A, double complex *B)
{
    double complex *R = malloc(sizeof(double complex) * (size_t)r * r);
    double T2 = 0.0;
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < r; ++j) {
            R[(size_t)i * r + j] = entry(ctx, i, j);
            T2 += creal(R[(size_t)i * r + j] * conj(R[(size_t)i * r + j]));
        }
    int k = 0;
    while (k < r) {
        double R2 = 0.0, m = 0.0;
        for (size_t e = 0; e < (size_t)r * r; ++e) {
            const double q = creal(R[e] * conj(R[e]));
            R2 += q;
            if (q > m) m = q;
        }
        if (R2 <= tol * tol * T2 || m == 0.0) break;
        size_t piv = 0;
        for (size_t e = 0; e < (size_t)r * r; ++e)
            if (creal(R[e] * conj(R[e])) >= (1.0 - 2e-9) * m) {
                piv = e;
                break;
            }
        const int pi = (int)(piv / r), pj = (int)(piv % r);
        const double complex pv = R[piv];
        for (int q = 0; q < r; ++q) {
            A[(size_t)k * r + q] = R[(size_t)q * r + pj];
            B[(size_t)k * r + q] = R[(size_t)pi * r + q] / pv;
        }
        for (int i = 0; i < r; ++i)
            for (int j = 0; j < r; ++j) R[(size_t)i * r + j] -= A[(size_t)k * r + i] * B[(size_t)k * r + j];
        ++k;
    }
    free(R);
    return k;
}

static double complex dense_entry(const void *ctx, int i, int j)
{
    const double *T = ((const double *const *)ctx)[0];
    const int r = (int)(intptr_t)((const void *const *)ctx)[1];
    return T[2 * ((size_t)i * r + j)] + I * T[2 * ((size_t)i * r + j) + 1];
}

int orc_aca(int r, const double *T, double tol, double *A, double *B)
{
    const void *ctx[2] = {T, (const void *)(intptr_t)r};
    return aca_factor(r, dense_entry, ctx, tol, (double complex *)A, (double complex *)B);
}

/* =========================================================================
 * Trees (Sec. 2.1, 2.2.1, 3.1)
 * ========================================================================= */
typedef struct {
    int64_t n;
    double corner[3];
    uint64_t *key;     /* sorted Morton keys                 */
    int64_t *perm;     /* sorted position -> user index      */
    double *P;         /* sorted coordinates, n x 3          */
    int64_t nbox[BITS + 1];
    int64_t *start[BITS + 1];   /* box b holds sorted points [start[b], start[b+1]) */
    int32_t *ijk[BITS + 1];     /* integer box coordinates, nbox x 3                */
    double *ctr[BITS + 1];      /* box centres, nbox x 3                            */
    int64_t *child[BITS + 1];   /* children of box b at l+1: [child[b], child[b+1]) */
    int built;                  /* deepest level built so far                       */
} tree_t;

typedef struct {
    int64_t n;
    int64_t *t, *s;
    int32_t *off;   /* far pairs: integer offset ijk_t - ijk_s */
} pairs_t;

struct orc_plan {
    int kernel;                /* ORC_LAPLACE or ORC_HELMHOLTZ */
    int dn;                    /* 1: the normal derivative at the targets (adjoint double layer) */
    int dl;                    /* 1: the normal derivative at the sources (double layer) */
    int grad;                  /* 1: the gradient at the targets, one axis at a time (axis; NXs = that axis) */
    int axis;
    double *NYs;               /* source normals in sorted order (dl plans) */
    double *NXs;               /* target normals in sorted order (dn plans) */
    double k, eps;
    orc_options opt;
    int empty;                 /* one of the sets is empty: v = 0 */
    int aligned;               /* both corners bitwise equal      */
    double d0, S;
    tree_t T[2];               /* 0 = targets X, 1 = sources Y    */
    int leaf;
    pairs_t far[BITS + 1];
    pairs_t near[BITS + 1];
    pairs_t early[BITS + 1];   /* per-pair leaf rule: near pairs of small boxes summed densely at level l */
    int method[BITS + 1];      /* 0 none, 1 Lagrange, 2 Gegenbauer */
    int order[BITS + 1];       /* r1 or L                          */
};

/* Morton key: 21 bits per axis interleaved, x in the highest bit of each triple (R12). */
static uint64_t interleave(int64_t qx, int64_t qy, int64_t qz)
{
    uint64_t key = 0;
    for (int b = 0; b < BITS; ++b) {
        key |= (uint64_t)((qx >> b) & 1) << (3 * b + 2);
        key |= (uint64_t)((qy >> b) & 1) << (3 * b + 1);
        key |= (uint64_t)((qz >> b) & 1) << (3 * b);
    }
    return key;
}

static void deinterleave(uint64_t prefix, int l, int32_t *ijk)
{
    int32_t i = 0, j = 0, m = 0;
    for (int b = 0; b < l; ++b) {
        i |= (int32_t)((prefix >> (3 * b + 2)) & 1) << b;
        j |= (int32_t)((prefix >> (3 * b + 1)) & 1) << b;
        m |= (int32_t)((prefix >> (3 * b)) & 1) << b;
    }
    ijk[0] = i;
    ijk[1] = j;
    ijk[2] = m;
}

static int64_t quantise(double p, double corner, double S)
{
    double t = (p - corner) * S;
    double f = floor(t);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)(QMAX - 1)) return QMAX - 1;
    return (int64_t)f;
}

typedef struct { uint64_t key; int64_t idx; } kv_t;

static int kv_cmp(const void *a, const void *b)
{
    const kv_t *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static void tree_build(tree_t *T, const double *P, int64_t n, const double corner[3], double S)
{
    T->n = n;
    memcpy(T->corner, corner, sizeof(double) * 3);
    kv_t *kv = malloc(sizeof(kv_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        kv[i].key = interleave(quantise(P[3 * i], corner[0], S), quantise(P[3 * i + 1], corner[1], S),
                               quantise(P[3 * i + 2], corner[2], S));
        kv[i].idx = i;
    }
    qsort(kv, (size_t)n, sizeof(kv_t), kv_cmp);   /* ascending key, ties by original index */
    T->key = malloc(sizeof(uint64_t) * (size_t)n);
    T->perm = malloc(sizeof(int64_t) * (size_t)n);
    T->P = malloc(sizeof(double) * 3 * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        T->key[i] = kv[i].key;
        T->perm[i] = kv[i].idx;
        memcpy(T->P + 3 * i, P + 3 * kv[i].idx, sizeof(double) * 3);
    }
    free(kv);
    T->built = -1;
}

/* Boxes of level l: the runs of equal key prefixes key >> 3(21 - l) in sorted order, with
 * integer coordinates and centres c = corner + (2i + 1) d_0 2^-(l+1) (Sec. 2.2.1, 3.1).
 * Also links level l-1 to its children. */
static void tree_level(tree_t *T, int l, double d0)
{
    int64_t n = T->n;
    int sh = 3 * (BITS - l);
    int64_t nb = 0;
    for (int64_t i = 0; i < n; ++i)
        if (i == 0 || (T->key[i] >> sh) != (T->key[i - 1] >> sh)) ++nb;
    T->nbox[l] = nb;
    T->start[l] = malloc(sizeof(int64_t) * (size_t)(nb + 1));
    T->ijk[l] = malloc(sizeof(int32_t) * 3 * (size_t)nb);
    T->ctr[l] = malloc(sizeof(double) * 3 * (size_t)nb);
    double h = ldexp(d0, -(l + 1));   /* half the box edge at level l */
    int64_t b = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (i == 0 || (T->key[i] >> sh) != (T->key[i - 1] >> sh)) {
            T->start[l][b] = i;
            deinterleave(T->key[i] >> sh, l, T->ijk[l] + 3 * b);
            for (int d = 0; d < 3; ++d)
                T->ctr[l][3 * b + d] = T->corner[d] + (double)(2 * T->ijk[l][3 * b + d] + 1) * h;
            ++b;
        }
    }
    T->start[l][nb] = n;
    T->child[l] = NULL;
    if (l > 0) {
        int64_t np = T->nbox[l - 1];
        T->child[l - 1] = malloc(sizeof(int64_t) * (size_t)(np + 1));
        int64_t c = 0;
        for (int64_t pb = 0; pb < np; ++pb) {
            while (T->start[l][c] < T->start[l - 1][pb]) ++c;
            T->child[l - 1][pb] = c;
        }
        T->child[l - 1][np] = nb;
    }
    T->built = l;
}

static void tree_free(tree_t *T)
{
    free(T->key);
    free(T->perm);
    free(T->P);
    for (int l = 0; l <= T->built; ++l) {
        free(T->start[l]);
        free(T->ijk[l]);
        free(T->ctr[l]);
        free(T->child[l]);
    }
}

/* =========================================================================
 * Plan: root cubes, trees, descent lists, stopping rule
 * ========================================================================= */
typedef struct { int64_t t, s; int32_t o[3]; } pr_t;

static int pr_cmp(const void *a, const void *b)
{
    const pr_t *x = a, *y = b;
    if (x->t != y->t) return x->t < y->t ? -1 : 1;
    return (x->s > y->s) - (x->s < y->s);
}

static void pairs_set(pairs_t *P, pr_t *v, int64_t n, int with_off)
{
    qsort(v, (size_t)n, sizeof(pr_t), pr_cmp);
    P->n = n;
    P->t = malloc(sizeof(int64_t) * (size_t)(n + 1));
    P->s = malloc(sizeof(int64_t) * (size_t)(n + 1));
    P->off = with_off ? malloc(sizeof(int32_t) * 3 * (size_t)(n + 1)) : NULL;
    for (int64_t i = 0; i < n; ++i) {
        P->t[i] = v[i].t;
        P->s[i] = v[i].s;
        if (with_off) memcpy(P->off + 3 * i, v[i].o, sizeof(int32_t) * 3);
    }
}

/* Admissibility (Sec. 2.2.2; reading R2): centres at max-norm distance >= 2 d_l. */
static int is_far(const orc_plan *p, int l, int64_t t, int64_t s)
{
    const tree_t *X = &p->T[0], *Y = &p->T[1];
    if (p->aligned) {
        int m = 0;
        for (int d = 0; d < 3; ++d) {
            int o = abs(X->ijk[l][3 * t + d] - Y->ijk[l][3 * s + d]);
            if (o > m) m = o;
        }
        return m >= 2;
    }
    double dl2 = 2.0 * ldexp(p->d0, -l), m = 0.0;
    for (int d = 0; d < 3; ++d) {
        double o = fabs(X->ctr[l][3 * t + d] - Y->ctr[l][3 * s + d]);
        if (o > m) m = o;
    }
    return m >= dl2;
}

orc_plan *orc_plan_create(const double *X, int64_t nx, const double *Y, int64_t ny,
                          int kernel, double k, double eps, const orc_options *opt)
{
    orc_plan *p = calloc(1, sizeof(orc_plan));
    p->grad = kernel == ORC_LAPLACE_GRAD || kernel == ORC_HELMHOLTZ_GRAD;
    p->dn = kernel == ORC_LAPLACE_DN || kernel == ORC_HELMHOLTZ_DN;
    p->dl = kernel == ORC_LAPLACE_DL || kernel == ORC_HELMHOLTZ_DL;
    kernel &= 1;
    p->kernel = kernel;
    p->k = k;
    p->eps = eps;
    p->opt.n_leaf = (opt && opt->n_leaf > 0) ? opt->n_leaf : 64;
    p->opt.kappa = (opt && opt->kappa > 0) ? opt->kappa : ORC_PI;
    p->opt.r1_override = opt ? opt->r1_override : 0;
    p->opt.max_level = (opt && opt->max_level > 0 && opt->max_level <= 20) ? opt->max_level : 20;
    p->opt.aca_tol = opt ? opt->aca_tol : 0.0;
    p->opt.adaptive = opt ? opt->adaptive : 0;
    if (opt)
        for (int l = 0; l < ORC_MAX_LEVELS; ++l) {
            p->opt.aca[l] = opt->aca[l];
            p->opt.grid_p[l] = opt->grid_p[l];
            p->opt.grid_w[l] = opt->grid_w[l];
            p->opt.grid_beta[l] = opt->grid_beta[l];
        }
    if (nx <= 0 || ny <= 0) {
        p->empty = 1;
        p->T[0].n = nx > 0 ? nx : 0;
        p->T[1].n = ny > 0 ? ny : 0;
        return p;
    }
    int maxlev = p->opt.max_level;

    /* Root cubes (Sec. 2.2.1; reading R1). */
    const double *PS[2] = {X, Y};
    int64_t NS[2] = {nx, ny};
    double lo[2][3], hi[2][3], d0 = 0.0;
    for (int e = 0; e < 2; ++e) {
        for (int d = 0; d < 3; ++d) {
            lo[e][d] = PS[e][d];
            hi[e][d] = PS[e][d];
        }
        for (int64_t i = 1; i < NS[e]; ++i)
            for (int d = 0; d < 3; ++d) {
                double v = PS[e][3 * i + d];
                if (v < lo[e][d]) lo[e][d] = v;
                if (v > hi[e][d]) hi[e][d] = v;
            }
        for (int d = 0; d < 3; ++d)
            if (hi[e][d] - lo[e][d] > d0) d0 = hi[e][d] - lo[e][d];
    }
    if (d0 == 0.0) d0 = 1.0;
    p->d0 = d0;
    p->S = (double)QMAX / d0;
    double corner[2][3];
    for (int e = 0; e < 2; ++e)
        for (int d = 0; d < 3; ++d) corner[e][d] = (lo[e][d] + hi[e][d]) * 0.5 - d0 * 0.5;
    p->aligned = memcmp(corner[0], corner[1], sizeof(double) * 3) == 0;

    /* Two octrees with the same cubic boxes at every level (Sec. 2.1). */
    for (int e = 0; e < 2; ++e) {
        tree_build(&p->T[e], PS[e], NS[e], corner[e], p->S);
        tree_level(&p->T[e], 0, d0);
    }
    if (p->dn || p->grad) {
        /* gradient plans: set per axis by orc_apply */
        p->NXs = calloc(3 * (size_t)nx, sizeof(double));
        if (!p->grad)
            for (int64_t i = 0; i < nx; ++i)
                for (int d = 0; d < 3; ++d) p->NXs[3 * i + d] = opt->target_normals[3 * p->T[0].perm[i] + d];
    }
    if (p->dl) {
        p->NYs = malloc(sizeof(double) * 3 * (size_t)ny);
        for (int64_t j = 0; j < ny; ++j)
            for (int d = 0; d < 3; ++d) p->NYs[3 * j + d] = opt->source_normals[3 * p->T[1].perm[j] + d];
    }

    /* Descent (Sec. 2.2.2, 2.2.4, 3.2): near_0 = {(root, root)}; the child pairs of every near
     * pair of level l-1 are split into far_l and near_l. */
    pr_t *root = malloc(sizeof(pr_t));
    root->t = 0;
    root->s = 0;
    pairs_set(&p->near[0], root, 1, 0);
    free(root);
    p->leaf = maxlev;
    for (int l = 1; l <= maxlev; ++l) {
        for (int e = 0; e < 2; ++e) tree_level(&p->T[e], l, d0);
        const pairs_t *pn = &p->near[l - 1];
        const tree_t *TX = &p->T[0], *TY = &p->T[1];
        int64_t cap = 0;
        for (int64_t i = 0; i < pn->n; ++i)
            cap += (TX->child[l - 1][pn->t[i] + 1] - TX->child[l - 1][pn->t[i]]) *
                   (TY->child[l - 1][pn->s[i] + 1] - TY->child[l - 1][pn->s[i]]);
        pr_t *vf = malloc(sizeof(pr_t) * (size_t)(cap + 1));
        pr_t *vn = malloc(sizeof(pr_t) * (size_t)(cap + 1));
        int64_t nf = 0, nn = 0;
        for (int64_t i = 0; i < pn->n; ++i)
            for (int64_t ct = TX->child[l - 1][pn->t[i]]; ct < TX->child[l - 1][pn->t[i] + 1]; ++ct)
                for (int64_t cs = TY->child[l - 1][pn->s[i]]; cs < TY->child[l - 1][pn->s[i] + 1]; ++cs) {
                    if (is_far(p, l, ct, cs)) {
                        vf[nf].t = ct;
                        vf[nf].s = cs;
                        for (int d = 0; d < 3; ++d)
                            vf[nf].o[d] = TX->ijk[l][3 * ct + d] - TY->ijk[l][3 * cs + d];
                        ++nf;
                    } else {
                        vn[nn].t = ct;
                        vn[nn].s = cs;
                        ++nn;
                    }
                }
        pairs_set(&p->far[l], vf, nf, 1);
        pairs_set(&p->near[l], vn, nn, 0);
        free(vf);
        free(vn);
        /* Stopping rule (Sec. 2.2.4; reading R4). */
        int64_t nb = p->T[0].nbox[l] + p->T[1].nbox[l];
        if (nn == 0 || nx + ny <= (int64_t)p->opt.n_leaf * nb || l == maxlev) {
            p->leaf = l;
            break;
        }
        /* Per-pair leaf rule (reading R22, beyond the paper's global rule): a near pair whose two boxes both hold
         * at most n_leaf points is not refined but summed densely at this level; the level is the leaf if no
         * near pair is left to refine. */
        if (p->opt.adaptive) {
            const pairs_t *N = &p->near[l];
            pr_t *ve = malloc(sizeof(pr_t) * (size_t)(N->n + 1)), *vr = malloc(sizeof(pr_t) * (size_t)(N->n + 1));
            int64_t ne = 0, nr = 0;
            for (int64_t i = 0; i < N->n; ++i) {
                const int64_t t = N->t[i], sb = N->s[i];
                const int64_t cx = TX->start[l][t + 1] - TX->start[l][t], cy = TY->start[l][sb + 1] - TY->start[l][sb];
                pr_t *dst = (cx <= p->opt.n_leaf && cy <= p->opt.n_leaf) ? &ve[ne++] : &vr[nr++];
                dst->t = t;
                dst->s = sb;
            }
            if (nr == 0) {
                free(ve);
                free(vr);
                p->leaf = l;
                break;
            }
            free(p->near[l].t);
            free(p->near[l].s);
            free(p->near[l].off);
            pairs_set(&p->near[l], vr, nr, 0);
            pairs_set(&p->early[l], ve, ne, 0);
            free(ve);
            free(vr);
        }
    }
    /* Compression form per level (Sec. 2.2.2-2.2.3; readings R5-R7). */
    for (int l = 1; l <= p->leaf; ++l) {
        double dl = ldexp(d0, -l);
        if (p->far[l].n == 0) continue;
        if (kernel == ORC_HELMHOLTZ && k * dl >= p->opt.kappa) {
            p->method[l] = 2;
            p->order[l] = orc_gegenbauer_rank(k, dl, eps);
        } else {
            p->method[l] = 1;
            int r1 = (int)ceil(log(1.0 / eps) / log(3.0 + sqrt(8.0)));
            if (kernel == ORC_HELMHOLTZ) r1 += (int)ceil(k * dl / 2.0);
            if (p->opt.r1_override > 0) r1 = p->opt.r1_override;
            if (r1 < 1) r1 = 1;
            p->order[l] = r1;
        }
    }
    return p;
}

void orc_plan_free(orc_plan *p)
{
    if (!p) return;
    free(p->NXs);
    free(p->NYs);
    if (!p->empty) {
        for (int e = 0; e < 2; ++e) tree_free(&p->T[e]);
        for (int l = 0; l <= BITS; ++l) {
            free(p->far[l].t);
            free(p->far[l].s);
            free(p->far[l].off);
            free(p->near[l].t);
            free(p->near[l].s);
            free(p->early[l].t);
            free(p->early[l].s);
        }
    }
    free(p);
}

/* =========================================================================
 * Apply
 * ========================================================================= */

/* CSR view of a sorted pair list by target. */
static int64_t *pairs_by_target(const pairs_t *P, int64_t ntgt)
{
    int64_t *ptr = calloc((size_t)(ntgt + 1), sizeof(int64_t));
    for (int64_t i = 0; i < P->n; ++i) ptr[P->t[i] + 1]++;
    for (int64_t t = 0; t < ntgt; ++t) ptr[t + 1] += ptr[t];
    return ptr;
}

/* Translation classes of a level: far pairs with equal integer offsets share one
 * transfer (proof of Prop. 1).  Classes are indexed through a dense window spanning
 * the offsets that occur at the level. */
typedef struct { int base[3], ext[3]; int32_t *id; int n; double (*r0)[3]; } classes_t;

static void classes_build(classes_t *C, const orc_plan *p, int l)
{
    double dl = ldexp(p->d0, -l);
    const pairs_t *F = &p->far[l];
    int hi[3];
    for (int d = 0; d < 3; ++d) {
        C->base[d] = F->n ? F->off[d] : 0;
        hi[d] = C->base[d];
    }
    for (int64_t i = 0; i < F->n; ++i)
        for (int d = 0; d < 3; ++d) {
            if (F->off[3 * i + d] < C->base[d]) C->base[d] = F->off[3 * i + d];
            if (F->off[3 * i + d] > hi[d]) hi[d] = F->off[3 * i + d];
        }
    for (int d = 0; d < 3; ++d) C->ext[d] = hi[d] - C->base[d] + 1;
    size_t nw = (size_t)C->ext[0] * C->ext[1] * C->ext[2];
    C->id = malloc(sizeof(int32_t) * nw);
    C->r0 = malloc(sizeof(double[3]) * nw);
    for (size_t i = 0; i < nw; ++i) C->id[i] = -1;
    C->n = 0;
    for (int64_t i = 0; i < F->n; ++i) {
        size_t idx = 0;
        for (int d = 0; d < 3; ++d) idx = idx * C->ext[d] + (F->off[3 * i + d] - C->base[d]);
        if (C->id[idx] < 0) {
            C->id[idx] = C->n;
            /* r0 = x0 - y0 = (corner_X - corner_Y) + o d_l */
            for (int d = 0; d < 3; ++d)
                C->r0[C->n][d] = (p->T[0].corner[d] - p->T[1].corner[d]) + (double)F->off[3 * i + d] * dl;
            C->n++;
        }
    }
}

static void classes_free(classes_t *C)
{
    free(C->id);
    free(C->r0);
}

static int class_of(const classes_t *C, const int32_t *o)
{
    size_t idx = 0;
    for (int d = 0; d < 3; ++d) idx = idx * C->ext[d] + (o[d] - C->base[d]);
    return C->id[idx];
}

/* Transfer-matrix entry of a translation class: T[(abc), (a'b'c')] = G(xi_t - xi_s), xi = c + (d_l/2)(t_a, t_b, t_c). */
typedef struct {
    const double *r0, *nodes;
    double dl, k;
    int r1, kernel;
} tentry_t;

static double complex class_entry(const void *ctx, int i, int j)
{
    const tentry_t *e = (const tentry_t *)ctx;
    const int r1 = e->r1;
    int ia[3] = {i / (r1 * r1), (i / r1) % r1, i % r1};
    int ja[3] = {j / (r1 * r1), (j / r1) % r1, j % r1};
    double dd[3];
    for (int d = 0; d < 3; ++d) dd[d] = e->r0[d] + 0.5 * e->dl * (e->nodes[ia[d]] - e->nodes[ja[d]]);
    return green(e->kernel, e->k, sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]));
}

/* Lagrange level (Sec. 2.2.2): v_t += L_X^T (sum_s T_{ts} (L_Y u_s)). */
static void level_lagrange(const orc_plan *p, int l, const double complex *u, double complex *v,
                           int64_t stride)
{
    const tree_t *TX = &p->T[0], *TY = &p->T[1];
    const pairs_t *F = &p->far[l];
    int r1 = p->order[l], r = r1 * r1 * r1;
    double dl = ldexp(p->d0, -l), nodes[64];
    orc_cheb_nodes(r1, nodes);
    int64_t nbx = TX->nbox[l], nby = TY->nbox[l];

    /* sources that take part in a far pair */
    char *need = calloc((size_t)nby, 1);
    for (int64_t i = 0; i < F->n; ++i) need[F->s[i]] = 1;

    /* interpolated source vectors u~_s = L_Y u_s (every stride-th point of a box when timing a sample) */
    double complex *ut = calloc((size_t)nby * r, sizeof(double complex));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < nby; ++s) {
        if (!need[s]) continue;
        double ex[64], ey[64], ez[64], gx[64], gy[64], gz[64];
        for (int64_t j = first_sample(TY->start[l][s], stride); j < TY->start[l][s + 1]; j += stride) {
            const double tx = 2.0 * (TY->P[3 * j] - TY->ctr[l][3 * s]) / dl;
            const double ty = 2.0 * (TY->P[3 * j + 1] - TY->ctr[l][3 * s + 1]) / dl;
            const double tz = 2.0 * (TY->P[3 * j + 2] - TY->ctr[l][3 * s + 2]) / dl;
            orc_lagrange_basis(r1, tx, ex);
            orc_lagrange_basis(r1, ty, ey);
            orc_lagrange_basis(r1, tz, ez);
            if (p->dl) {
                /* G(x, y) ~ sum_nodes G(x, y_node) L_node(y): its derivative along n_y weights the nodes by
                 * n_y . grad L_node(y), d/dy of l(2 (y - c) / d_l) being (2 / d_l) l' */
                const double *n = p->NYs + 3 * j;
                orc_lagrange_basis_deriv(r1, tx, gx);
                orc_lagrange_basis_deriv(r1, ty, gy);
                orc_lagrange_basis_deriv(r1, tz, gz);
                for (int a = 0; a < r1; ++a)
                    for (int b = 0; b < r1; ++b)
                        for (int c = 0; c < r1; ++c) {
                            const double g = n[0] * gx[a] * ey[b] * ez[c] + n[1] * ex[a] * gy[b] * ez[c] +
                                             n[2] * ex[a] * ey[b] * gz[c];
                            ut[s * r + (a * r1 + b) * r1 + c] += (2.0 / dl) * g * u[j];
                        }
                continue;
            }
            for (int a = 0; a < r1; ++a)
                for (int b = 0; b < r1; ++b)
                    for (int c = 0; c < r1; ++c) ut[s * r + (a * r1 + b) * r1 + c] += ex[a] * ey[b] * ez[c] * u[j];
        }
    }

    /* transfer matrices T[(abc),(a'b'c')] = G(xi_t - xi_s), one per translation; with ACA (eq. ffmACAmatvec)
     * each is kept as its factors A (r x k_c), B (r x k_c) instead */
    classes_t C;
    classes_build(&C, p, l);
    const int use_aca = p->opt.aca_tol > 0.0 && p->opt.aca[l];
    double complex *Tm = NULL, **Af = NULL, **Bf = NULL;
    int *kc = NULL;
    if (!use_aca) {
        Tm = malloc(sizeof(double complex) * (size_t)C.n * r * r);
#pragma omp parallel for schedule(dynamic, 1)
        for (int c = 0; c < C.n; ++c) {
            tentry_t te = {C.r0[c], nodes, dl, p->k, r1, p->kernel};
            for (int i = 0; i < r; ++i)
                for (int j = 0; j < r; ++j) Tm[((size_t)c * r + i) * r + j] = class_entry(&te, i, j);
        }
    } else {
        Af = calloc((size_t)C.n, sizeof(double complex *));
        Bf = calloc((size_t)C.n, sizeof(double complex *));
        kc = calloc((size_t)C.n, sizeof(int));
#pragma omp parallel for schedule(dynamic, 1)
        for (int c = 0; c < C.n; ++c) {
            tentry_t te = {C.r0[c], nodes, dl, p->k, r1, p->kernel};
            double complex *A = malloc(sizeof(double complex) * (size_t)r * r);
            double complex *B = malloc(sizeof(double complex) * (size_t)r * r);
            kc[c] = aca_factor(r, class_entry, &te, p->opt.aca_tol, A, B);
            Af[c] = A;
            Bf[c] = B;
        }
    }

    /* v~_t = sum_{s in far(t)} T_ts u~_s ;  v_i += sum L_i(x) v~_t */
    int64_t *ptr = pairs_by_target(F, nbx);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nbx; ++t) {
        if (ptr[t] == ptr[t + 1]) continue;
        double complex *vt = calloc((size_t)r, sizeof(double complex));
        for (int64_t e = ptr[t]; e < ptr[t + 1]; ++e) {
            const int c = class_of(&C, F->off + 3 * e);
            const double complex *us = ut + F->s[e] * r;
            if (use_aca) {
                /* v~ += A (B^T u~) */
                for (int q = 0; q < kc[c]; ++q) {
                    double complex z = 0.0;
                    for (int j = 0; j < r; ++j) z += Bf[c][(size_t)q * r + j] * us[j];
                    for (int i = 0; i < r; ++i) vt[i] += Af[c][(size_t)q * r + i] * z;
                }
                continue;
            }
            const double complex *Tc = Tm + (size_t)c * r * r;
            for (int i = 0; i < r; ++i) {
                double complex acc = 0.0;
                for (int j = 0; j < r; ++j) acc += Tc[i * r + j] * us[j];
                vt[i] += acc;
            }
        }
        double ex[64], ey[64], ez[64], dx[64], dy[64], dz[64];
        for (int64_t i = first_sample(TX->start[l][t], stride); i < TX->start[l][t + 1]; i += stride) {
            const double tx = 2.0 * (TX->P[3 * i] - TX->ctr[l][3 * t]) / dl;
            const double ty = 2.0 * (TX->P[3 * i + 1] - TX->ctr[l][3 * t + 1]) / dl;
            const double tz = 2.0 * (TX->P[3 * i + 2] - TX->ctr[l][3 * t + 2]) / dl;
            orc_lagrange_basis(r1, tx, ex);
            orc_lagrange_basis(r1, ty, ey);
            orc_lagrange_basis(r1, tz, ez);
            double complex acc = 0.0;
            if (p->dn || p->grad) {
                /* n . grad of the interpolant; d/dx of l(2 (x - c) / d_l) is (2 / d_l) l' */
                const double *n = p->NXs + 3 * i;
                orc_lagrange_basis_deriv(r1, tx, dx);
                orc_lagrange_basis_deriv(r1, ty, dy);
                orc_lagrange_basis_deriv(r1, tz, dz);
                for (int a = 0; a < r1; ++a)
                    for (int b = 0; b < r1; ++b)
                        for (int c = 0; c < r1; ++c) {
                            const double g = n[0] * dx[a] * ey[b] * ez[c] + n[1] * ex[a] * dy[b] * ez[c] +
                                             n[2] * ex[a] * ey[b] * dz[c];
                            acc += (2.0 / dl) * g * vt[(a * r1 + b) * r1 + c];
                        }
            } else {
                for (int a = 0; a < r1; ++a)
                    for (int b = 0; b < r1; ++b)
                        for (int c = 0; c < r1; ++c) acc += ex[a] * ey[b] * ez[c] * vt[(a * r1 + b) * r1 + c];
            }
            v[i] += acc;
        }
        free(vt);
    }
    free(ptr);
    free(Tm);
    if (use_aca) {
        for (int c = 0; c < C.n; ++c) {
            free(Af[c]);
            free(Bf[c]);
        }
        free(Af);
        free(Bf);
        free(kc);
    }
    classes_free(&C);
    free(ut);
    free(need);
}

int orc_aca_ranks(const orc_plan *p, int l, double tol, int32_t *off, int32_t *ranks)
{
    if (p->empty || l < 1 || l > p->leaf || p->method[l] != 1) return 0;
    classes_t C;
    classes_build(&C, p, l);
    int r1 = p->order[l], r = r1 * r1 * r1;
    double dl = ldexp(p->d0, -l), nodes[64];
    orc_cheb_nodes(r1, nodes);
    const pairs_t *F = &p->far[l];
    for (int64_t i = 0; i < F->n; ++i) {
        const int c = class_of(&C, F->off + 3 * i);
        for (int d = 0; d < 3; ++d) off[3 * c + d] = F->off[3 * i + d];
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < C.n; ++c) {
        tentry_t te = {C.r0[c], nodes, dl, p->k, r1, p->kernel};
        double complex *A = malloc(sizeof(double complex) * (size_t)r * r);
        double complex *B = malloc(sizeof(double complex) * (size_t)r * r);
        ranks[c] = aca_factor(r, class_entry, &te, tol, A, B);
        free(A);
        free(B);
    }
    const int n = C.n;
    classes_free(&C);
    return n;
}

/* Gegenbauer level (Sec. 2.2.3): v = F_{s->X} (D (F_{Y->s} u)) in box-centred coordinates (R9). */
static void level_gegenbauer(const orc_plan *p, int l, const double complex *u, double complex *v,
                             int64_t stride)
{
    const tree_t *TX = &p->T[0], *TY = &p->T[1];
    const pairs_t *F = &p->far[l];
    int L = p->order[l];
    double k = p->k;
    int64_t nq = 2 * (int64_t)L * (L + 1);
    double *s = malloc(sizeof(double) * 3 * nq), *w = malloc(sizeof(double) * nq);
    orc_sphere_quadrature(L, s, w);
    int64_t nbx = TX->nbox[l], nby = TY->nbox[l];

    /* sources that take part in a far pair */
    char *need = calloc((size_t)nby, 1);
    int64_t *ptr = pairs_by_target(F, nbx);
    for (int64_t i = 0; i < F->n; ++i) need[F->s[i]] = 1;

    /* grid form of the transforms at this level (R16-R18), else the direct sums */
    /* grid form of the transforms where asked */
    const int grid = p->opt.grid_p[l] > 0;
    gridlev_t gl;
    if (grid) {
        int gp = p->opt.grid_p[l], gw = p->opt.grid_w[l];
        gridlev_init(&gl, gp, gw, p->opt.grid_beta[l], ldexp(p->d0, -l) / (double)(gp - 1 - gw), k, L);
    }

    /* forward transform u~_s(q) = sum_j e^{-ik s_q.(y_j - c_s)} u_j (every stride-th point of a box when timing
     * a sample) */
    double complex *ut = calloc((size_t)nby * nq, sizeof(double complex));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < nby; ++b) {
        if (!need[b]) continue;
        const double *c = TY->ctr[l] + 3 * b;
        if (grid) {
            int64_t j0 = first_sample(TY->start[l][b], stride);
            int64_t nb = TY->start[l][b + 1] > j0 ? (TY->start[l][b + 1] - j0 + stride - 1) / stride : 0;
            double *yr = malloc(sizeof(double) * 3 * (size_t)(nb + 1));
            double complex *ub = malloc(sizeof(double complex) * (size_t)(nb + 1));
            for (int64_t j = 0; j < nb; ++j)
                for (int d = 0; d < 3; ++d) yr[3 * j + d] = TY->P[3 * (j0 + j * stride) + d] - c[d];
            if (p->dl) {
                /* n . grad_y: -ik sum_c s_c (the grid form's source transform of the density u n_c) */
                double complex *uc = calloc((size_t)nq, sizeof(double complex));
                for (int ax = 0; ax < 3; ++ax) {
                    for (int64_t j = 0; j < nb; ++j) ub[j] = u[j0 + j * stride] * p->NYs[3 * (j0 + j * stride) + ax];
                    for (int64_t q = 0; q < nq; ++q) uc[q] = 0.0;
                    grid_fwd(&gl, yr, ub, nb, uc);
                    for (int64_t q = 0; q < nq; ++q) ut[b * nq + q] += -I * k * s[3 * q + ax] * uc[q];
                }
                free(uc);
            } else {
                for (int64_t j = 0; j < nb; ++j) ub[j] = u[j0 + j * stride];
                grid_fwd(&gl, yr, ub, nb, ut + b * nq);
            }
            free(yr);
            free(ub);
            continue;
        }
        for (int64_t j = first_sample(TY->start[l][b], stride); j < TY->start[l][b + 1]; j += stride) {
            double y0 = TY->P[3 * j] - c[0], y1 = TY->P[3 * j + 1] - c[1], y2 = TY->P[3 * j + 2] - c[2];
            if (p->dl) {
                /* n . grad_y e^{-ik s.(y - c)} = -ik (s . n) e^{-ik s.(y - c)} */
                const double *n = p->NYs + 3 * j;
                for (int64_t q = 0; q < nq; ++q)
                    ut[b * nq + q] += -I * k * (s[3 * q] * n[0] + s[3 * q + 1] * n[1] + s[3 * q + 2] * n[2]) *
                                      cexp(-I * k * (s[3 * q] * y0 + s[3 * q + 1] * y1 + s[3 * q + 2] * y2)) * u[j];
                continue;
            }
            for (int64_t q = 0; q < nq; ++q)
                ut[b * nq + q] += cexp(-I * k * (s[3 * q] * y0 + s[3 * q + 1] * y1 + s[3 * q + 2] * y2)) * u[j];
        }
    }

    /* diagonal transfer per translation class */
    classes_t C;
    classes_build(&C, p, l);
    double complex *D = malloc(sizeof(double complex) * (size_t)C.n * nq);
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < C.n; ++c) gegenbauer_diag_q(L, k, C.r0[c], s, w, nq, D + (size_t)c * nq);

    /* v~_t(q) = sum_s D_ts(q) u~_s(q);  v_i += sum_q e^{ik s_q.(x_i - c_t)} v~_t(q) */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nbx; ++t) {
        if (ptr[t] == ptr[t + 1]) continue;
        double complex *vt = calloc((size_t)nq, sizeof(double complex));
        for (int64_t e = ptr[t]; e < ptr[t + 1]; ++e) {
            const double complex *Dc = D + (size_t)class_of(&C, F->off + 3 * e) * nq;
            const double complex *us = ut + F->s[e] * nq;
            for (int64_t q = 0; q < nq; ++q) vt[q] += Dc[q] * us[q];
        }
        /* gradient, component axis: d/dx_axis e^{ik s.(x - c)} = ik s_axis e^{ik s.(x - c)}, so the target
         * transform (direct or grid) of ik s_axis v~ */
        if (p->grad)
            for (int64_t q = 0; q < nq; ++q) vt[q] *= I * k * s[3 * q + p->axis];
        const double *c = TX->ctr[l] + 3 * t;
        if (grid) {
            int64_t i0 = first_sample(TX->start[l][t], stride);
            int64_t nt = TX->start[l][t + 1] > i0 ? (TX->start[l][t + 1] - i0 + stride - 1) / stride : 0;
            double *xr = malloc(sizeof(double) * 3 * (size_t)(nt + 1));
            double complex *vb = calloc((size_t)(nt + 1), sizeof(double complex));
            for (int64_t i = 0; i < nt; ++i)
                for (int d = 0; d < 3; ++d) xr[3 * i + d] = TX->P[3 * (i0 + i * stride) + d] - c[d];
            if (p->dn) {
                /* n . grad: the grid form's target transforms of ik s_c v~, c = 0, 1, 2, combined with n_c */
                double complex *vc = malloc(sizeof(double complex) * (size_t)nq);
                for (int ax = 0; ax < 3; ++ax) {
                    for (int64_t q = 0; q < nq; ++q) vc[q] = I * k * s[3 * q + ax] * vt[q];
                    for (int64_t i = 0; i < nt; ++i) vb[i] = 0.0;
                    grid_bwd(&gl, vc, xr, nt, vb);
                    for (int64_t i = 0; i < nt; ++i) v[i0 + i * stride] += p->NXs[3 * (i0 + i * stride) + ax] * vb[i];
                }
                free(vc);
            } else {
                grid_bwd(&gl, vt, xr, nt, vb);
                for (int64_t i = 0; i < nt; ++i) v[i0 + i * stride] += vb[i];
            }
            free(xr);
            free(vb);
            free(vt);
            continue;
        }
        for (int64_t i = first_sample(TX->start[l][t], stride); i < TX->start[l][t + 1]; i += stride) {
            double x0 = TX->P[3 * i] - c[0], x1 = TX->P[3 * i + 1] - c[1], x2 = TX->P[3 * i + 2] - c[2];
            double complex acc = 0.0;
            if (p->dn) {
                /* n . grad_x e^{ik s.(x - c)} = ik (s . n) e^{ik s.(x - c)} */
                const double *n = p->NXs + 3 * i;
                for (int64_t q = 0; q < nq; ++q)
                    acc += I * k * (s[3 * q] * n[0] + s[3 * q + 1] * n[1] + s[3 * q + 2] * n[2]) *
                           cexp(I * k * (s[3 * q] * x0 + s[3 * q + 1] * x1 + s[3 * q + 2] * x2)) * vt[q];
            } else {
                for (int64_t q = 0; q < nq; ++q)
                    acc += cexp(I * k * (s[3 * q] * x0 + s[3 * q + 1] * x1 + s[3 * q + 2] * x2)) * vt[q];
            }
            v[i] += acc;
        }
        free(vt);
    }
    if (grid) gridlev_free(&gl);
    free(D);
    classes_free(&C);
    free(ut);
    free(ptr);
    free(need);
    free(s);
    free(w);
}

/* Dense remainder (Sec. 2.2.4): the near pairs of the leaf, and those the per-pair rule stopped earlier
 * (level l < leaf, list early). */
static void near_pairs_sum(const orc_plan *p, int l, const pairs_t *N, const double complex *u, double complex *v,
                           int64_t stride);

static void near_field(const orc_plan *p, const double complex *u, double complex *v, int64_t stride)
{
    for (int l = 1; l < p->leaf; ++l)
        if (p->early[l].n) near_pairs_sum(p, l, &p->early[l], u, v, stride);
    near_pairs_sum(p, p->leaf, &p->near[p->leaf], u, v, stride);
}

static void near_pairs_sum(const orc_plan *p, int l, const pairs_t *N, const double complex *u, double complex *v,
                           int64_t stride)
{
    const tree_t *TX = &p->T[0], *TY = &p->T[1];
    int64_t nbx = TX->nbox[l];
    int64_t *ptr = pairs_by_target(N, nbx);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < nbx; ++t) {
        for (int64_t e = ptr[t]; e < ptr[t + 1]; ++e) {
            int64_t sb = N->s[e];
            for (int64_t i = first_sample(TX->start[l][t], stride); i < TX->start[l][t + 1]; i += stride) {
                double complex acc = 0.0;
                for (int64_t j = TY->start[l][sb]; j < TY->start[l][sb + 1]; ++j) {
                    double dx = TX->P[3 * i] - TY->P[3 * j], dy = TX->P[3 * i + 1] - TY->P[3 * j + 1],
                           dz = TX->P[3 * i + 2] - TY->P[3 * j + 2];
                    double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 == 0.0) continue;   /* R11 */
                    if (p->dn || p->grad) {
                        const double d[3] = {dx, dy, dz};
                        acc += green_dn(p->kernel, p->k, d, p->NXs + 3 * i) * u[j];
                    } else if (p->dl) {
                        const double d[3] = {dx, dy, dz};
                        acc += green_dl(p->kernel, p->k, d, p->NYs + 3 * j) * u[j];
                    } else {
                        acc += green(p->kernel, p->k, sqrt(r2)) * u[j];
                    }
                }
                v[i] += acc;
            }
        }
    }
    free(ptr);
}

/* the product in tree order: vs += every level's far pairs, in order (Sec. 2.2), then the near field */
static void apply_sorted(const orc_plan *p, const double complex *u, double complex *vs, int64_t stride)
{
    for (int l = 1; l <= p->leaf; ++l) {
        if (p->method[l] == 1) level_lagrange(p, l, u, vs, stride);
        else if (p->method[l] == 2) level_gegenbauer(p, l, u, vs, stride);
    }
    near_field(p, u, vs, stride);
}

void orc_apply(orc_plan *p, const double *wu, double *v, int64_t stride)
{
    if (stride < 1) stride = 1;
    int64_t nx = p->T[0].n, ny = p->T[1].n;
    const int ncomp = p->grad ? 3 : 1;
    memset(v, 0, sizeof(double) * 2 * (size_t)nx * ncomp);
    if (p->empty) return;
    /* permute the input into source tree order */
    double complex *u = malloc(sizeof(double complex) * (size_t)ny);
    for (int64_t j = 0; j < ny; ++j) u[j] = cload(wu, p->T[1].perm[j]);
    double complex *vs = malloc(sizeof(double complex) * (size_t)(nx > 0 ? nx : 1));
    for (int c = 0; c < ncomp; ++c) {
        /* gradient: component c is the derivative along axis c (the normal derivative with n = e_c at Lagrange
         * levels and in the near field) */
        if (p->grad) {
            p->axis = c;
            for (int64_t i = 0; i < nx; ++i)
                for (int d = 0; d < 3; ++d) p->NXs[3 * i + d] = d == c ? 1.0 : 0.0;
        }
        for (int64_t i = 0; i < nx; ++i) vs[i] = 0.0;
        apply_sorted(p, u, vs, stride);
        /* back to the user's target order */
        for (int64_t i = 0; i < nx; ++i) {
            const int64_t o = ncomp * p->T[0].perm[i] + c;
            v[2 * o] = creal(vs[i]);
            v[2 * o + 1] = cimag(vs[i]);
        }
    }
    free(vs);
    free(u);
}

/* =========================================================================
 * Queries
 * ========================================================================= */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* memcpy of n bytes that accepts an absent source when there is nothing to copy (empty plans keep no arrays) */
static void copy_out(void *dst, const void *src, size_t n)
{
    if (n > 0 && src) memcpy(dst, src, n);
}

int orc_leaf(const orc_plan *p) { return p->empty ? 0 : p->leaf; }
double orc_d0(const orc_plan *p) { return p->d0; }
void orc_corner(const orc_plan *p, int set, double *c3) { memcpy(c3, p->T[set].corner, sizeof(double) * 3); }
int64_t orc_npoints(const orc_plan *p, int set) { return p->T[set].n; }
void orc_keys(const orc_plan *p, int set, uint64_t *keys)
{
    copy_out(keys, p->T[set].key, sizeof(uint64_t) * (size_t)p->T[set].n);
}
void orc_perm(const orc_plan *p, int set, int64_t *perm)
{
    copy_out(perm, p->T[set].perm, sizeof(int64_t) * (size_t)p->T[set].n);
}
int64_t orc_nbox(const orc_plan *p, int set, int l) { return p->empty ? 0 : p->T[set].nbox[l]; }
void orc_box_start(const orc_plan *p, int set, int l, int64_t *start)
{
    if (p->empty) {
        start[0] = 0;
        return;
    }
    copy_out(start, p->T[set].start[l], sizeof(int64_t) * (size_t)(p->T[set].nbox[l] + 1));
}
void orc_box_ijk(const orc_plan *p, int set, int l, int32_t *ijk)
{
    if (!p->empty) copy_out(ijk, p->T[set].ijk[l], sizeof(int32_t) * 3 * (size_t)p->T[set].nbox[l]);
}
void orc_box_centre(const orc_plan *p, int set, int l, double *c)
{
    if (!p->empty) copy_out(c, p->T[set].ctr[l], sizeof(double) * 3 * (size_t)p->T[set].nbox[l]);
}
int64_t orc_nfar(const orc_plan *p, int l) { return (p->empty || l > p->leaf) ? 0 : p->far[l].n; }
void orc_far(const orc_plan *p, int l, int64_t *t, int64_t *s, int32_t *off)
{
    const pairs_t *F = &p->far[l];
    copy_out(t, F->t, sizeof(int64_t) * (size_t)F->n);
    copy_out(s, F->s, sizeof(int64_t) * (size_t)F->n);
    copy_out(off, F->off, sizeof(int32_t) * 3 * (size_t)F->n);
}
int64_t orc_nearly(const orc_plan *p, int l) { return (p->empty || l > p->leaf) ? 0 : p->early[l].n; }
void orc_early(const orc_plan *p, int l, int64_t *t, int64_t *s)
{
    copy_out(t, p->early[l].t, sizeof(int64_t) * (size_t)p->early[l].n);
    copy_out(s, p->early[l].s, sizeof(int64_t) * (size_t)p->early[l].n);
}
int64_t orc_nnear(const orc_plan *p, int l) { return (p->empty || l > p->leaf) ? 0 : p->near[l].n; }
void orc_near(const orc_plan *p, int l, int64_t *t, int64_t *s)
{
    const pairs_t *N = &p->near[l];
    copy_out(t, N->t, sizeof(int64_t) * (size_t)N->n);
    copy_out(s, N->s, sizeof(int64_t) * (size_t)N->n);
}
int orc_level_method(const orc_plan *p, int l) { return (p->empty || l > p->leaf) ? 0 : p->method[l]; }
int orc_level_order(const orc_plan *p, int l) { return (p->empty || l > p->leaf) ? 0 : p->order[l]; }
