/*
 * Driver for a host-sanitizer build of the oracle (AddressSanitizer + UndefinedBehaviorSanitizer, gcc): it
 * runs every entry point of oracle/ffm_oracle.c on small synthetic inputs (both kernels, Lagrange and
 * Gegenbauer levels, direct and grid transforms, ACA, the normal derivatives at the target and at the source,
 * the gradient, the per-pair leaf rule, distinct and empty sets) and checks that the products are finite and agree with the dense definition.
 * Any out-of-bounds access, use after free, leak or undefined operation aborts the run.
 *
 * Test infrastructure: built and run by tests/test_oracle_sanitize.py only.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ffm_oracle.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

static double unif(void) {   /* splitmix64 -> [0, 1) */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
}

static double gauss(void) {
    const double a = unif() + 1e-300, b = unif();
    return sqrt(-2.0 * log(a)) * cos(2.0 * M_PI * b);
}

static void sphere(double *X, int64_t n, double r, double cx) {
    for (int64_t i = 0; i < n; ++i) {
        double v[3] = {gauss(), gauss(), gauss()};
        const double s = r / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        X[3 * i] = v[0] * s + cx;
        X[3 * i + 1] = v[1] * s;
        X[3 * i + 2] = v[2] * s;
    }
}

static void input(double *wu, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        wu[2 * i] = gauss() / (double)n;
        wu[2 * i + 1] = gauss() / (double)n;
    }
}

static int failures = 0;

/* relative L2 distance of the product rows from the dense rows */
static void check(const char *name, const double *v, const double *d, const int64_t *rows, int64_t nr, double tol) {
    double num = 0.0, den = 0.0;
    for (int64_t a = 0; a < nr; ++a) {
        const double *x = v + 2 * rows[a], *y = d + 2 * a;
        if (!isfinite(x[0]) || !isfinite(x[1])) {
            printf("%s: non-finite product at row %lld\n", name, (long long)rows[a]);
            ++failures;
            return;
        }
        num += (x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]);
        den += y[0] * y[0] + y[1] * y[1];
    }
    const double e = sqrt(num / (den > 0 ? den : 1.0));
    printf("%s: %.3e (bound %.1e)\n", name, e, tol);
    if (!(e <= tol)) ++failures;
}

static void run(const char *name, const double *X, int64_t nx, const double *Y, int64_t ny, int kernel, double k,
                double eps, const orc_options *opt, const double *normals) {
    const int grad = kernel == ORC_LAPLACE_GRAD || kernel == ORC_HELMHOLTZ_GRAD;
    const int nc = grad ? 3 : 1;
    double *wu = malloc(sizeof(double) * 2 * (size_t)(ny > 0 ? ny : 1));
    double *v = malloc(sizeof(double) * 2 * (size_t)nc * (nx > 0 ? nx : 1));
    input(wu, ny);
    orc_plan *p = orc_plan_create(X, nx, Y, ny, kernel, k, eps, opt);
    if (!p) {
        printf("%s: plan failed\n", name);
        ++failures;
        free(wu);
        free(v);
        return;
    }
    orc_apply(p, wu, v, 1);
    /* queries over every level */
    const int leaf = orc_leaf(p);
    for (int l = 0; l <= leaf; ++l) {
        for (int set = 0; set < 2; ++set) {
            const int64_t nb = orc_nbox(p, set, l);
            int64_t *st = malloc(sizeof(int64_t) * (size_t)(nb + 1));
            int32_t *ijk = malloc(sizeof(int32_t) * 3 * (size_t)(nb > 0 ? nb : 1));
            double *c = malloc(sizeof(double) * 3 * (size_t)(nb > 0 ? nb : 1));
            orc_box_start(p, set, l, st);
            orc_box_ijk(p, set, l, ijk);
            orc_box_centre(p, set, l, c);
            free(st);
            free(ijk);
            free(c);
        }
        const int64_t nf = orc_nfar(p, l), nn = orc_nnear(p, l), ne = orc_nearly(p, l);
        int64_t *t = malloc(sizeof(int64_t) * (size_t)(nf + nn + ne + 1));
        int64_t *s = malloc(sizeof(int64_t) * (size_t)(nf + nn + ne + 1));
        int32_t *off = malloc(sizeof(int32_t) * 3 * (size_t)(nf + 1));
        if (nf) orc_far(p, l, t, s, off);
        if (nn) orc_near(p, l, t, s);
        if (ne) orc_early(p, l, t, s);
        free(t);
        free(s);
        free(off);
        (void)orc_level_method(p, l);
        (void)orc_level_order(p, l);
    }
    if (nx > 0 && ny > 0) {
        const int64_t nr = nx < 40 ? nx : 40;
        int64_t *rows = malloc(sizeof(int64_t) * (size_t)nr);
        for (int64_t a = 0; a < nr; ++a) rows[a] = (a * 7919) % nx;
        double *d = malloc(sizeof(double) * 2 * (size_t)nr * nc);
        if (grad) {
            /* component by component: rows 3 r + c of the product against entries 3 a + c */
            int64_t *r3 = malloc(sizeof(int64_t) * 3 * (size_t)nr);
            for (int64_t a = 0; a < nr; ++a)
                for (int c = 0; c < 3; ++c) r3[3 * a + c] = 3 * rows[a] + c;
            orc_dense_rows_grad(X, Y, ny, wu, kernel & 1, k, rows, nr, d);
            check(name, v, d, r3, 3 * nr, eps);
            free(r3);
            free(rows);
            free(d);
            orc_plan_free(p);
            free(wu);
            free(v);
            return;
        }
        if (kernel == ORC_LAPLACE_DL || kernel == ORC_HELMHOLTZ_DL)
            orc_dense_rows_dl(X, Y, ny, wu, kernel & 1, k, normals, rows, nr, d);
        else if (kernel >= ORC_LAPLACE_DN)
            orc_dense_rows_dn(X, Y, ny, wu, kernel & 1, k, normals, rows, nr, d);
        else
            orc_dense_rows(X, Y, ny, wu, kernel, k, rows, nr, d);
        check(name, v, d, rows, nr, eps);
        free(rows);
        free(d);
    }
    orc_plan_free(p);
    free(wu);
    free(v);
}

int main(void) {
    const int64_t n = 3000;
    double *X = malloc(sizeof(double) * 3 * n), *Y = malloc(sizeof(double) * 3 * 2000);
    double *N = malloc(sizeof(double) * 3 * n);
    sphere(X, n, 1.0, 0.0);
    sphere(Y, 2000, 0.9, 0.05);
    /* unit normals in random directions (radial normals on a sphere make n . grad G cancel for close pairs,
     * which amplifies the relative error of the interpolated derivative; that case is not a sanitizer matter) */
    for (int64_t i = 0; i < n; ++i) {
        double v[3] = {gauss(), gauss(), gauss()};
        const double s = 1.0 / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        for (int c = 0; c < 3; ++c) N[3 * i + c] = v[c] * s;
    }
    orc_options o;

    memset(&o, 0, sizeof(o));
    run("laplace", X, n, X, n, ORC_LAPLACE, 0.0, 1e-3, &o, NULL);
    run("helmholtz k=30", X, n, X, n, ORC_HELMHOLTZ, 30.0, 1e-3, &o, NULL);
    run("helmholtz distinct sets", X, n, Y, 2000, ORC_HELMHOLTZ, 12.0, 1e-3, &o, NULL);
    run("empty sources", X, 300, Y, 0, ORC_LAPLACE, 0.0, 1e-3, &o, NULL);
    run("empty targets", X, 0, Y, 200, ORC_HELMHOLTZ, 3.0, 1e-3, &o, NULL);

    /* ACA at every Lagrange level */
    memset(&o, 0, sizeof(o));
    o.aca_tol = 1e-4 / 4.0;
    for (int l = 0; l < ORC_MAX_LEVELS; ++l) o.aca[l] = 1;
    run("laplace aca", X, n, X, n, ORC_LAPLACE, 0.0, 1e-4, &o, NULL);

    /* grid form at level 2 of a Helmholtz plan (kd = 30 / 2 at level 1 ... Gegenbauer levels from 1) */
    memset(&o, 0, sizeof(o));
    o.grid_p[2] = 32;
    o.grid_w[2] = 6;
    o.grid_beta[2] = 2.3 * 6;
    run("helmholtz grid level 2", X, n, X, n, ORC_HELMHOLTZ, 30.0, 1e-3, &o, NULL);

    /* normal derivative at the target */
    memset(&o, 0, sizeof(o));
    o.target_normals = N;
    run("laplace dn", X, n, X, n, ORC_LAPLACE_DN, 0.0, 1e-3, &o, N);
    run("helmholtz dn", X, n, X, n, ORC_HELMHOLTZ_DN, 25.0, 1e-3, &o, N);

    /* gradient at the target */
    memset(&o, 0, sizeof(o));
    run("laplace grad", X, n, X, n, ORC_LAPLACE_GRAD, 0.0, 1e-3, &o, NULL);
    run("helmholtz grad distinct sets", X, n, Y, 2000, ORC_HELMHOLTZ_GRAD, 20.0, 1e-3, &o, NULL);

    /* normal derivative at the source (double layer) */
    memset(&o, 0, sizeof(o));
    o.source_normals = N;
    run("laplace dl", X, n, X, n, ORC_LAPLACE_DL, 0.0, 1e-3, &o, N);
    run("helmholtz dl", X, n, X, n, ORC_HELMHOLTZ_DL, 25.0, 1e-3, &o, N);

    /* per-pair leaf rule on a sphere with a dense cluster */
    double *Z = malloc(sizeof(double) * 3 * n);
    sphere(Z, 2000, 1.0, 0.0);
    for (int64_t i = 2000; i < n; ++i)
        for (int c = 0; c < 3; ++c) Z[3 * i + c] = 0.3 + 0.05 * unif();
    memset(&o, 0, sizeof(o));
    o.adaptive = 1;
    run("laplace adaptive", Z, n, Z, n, ORC_LAPLACE, 0.0, 1e-3, &o, NULL);

    /* building blocks */
    double gx[16], gw[16], P[12], h[24], ell[8], del[8], t[8];
    orc_gauss_legendre(16, gx, gw);
    orc_legendre_p(11, 0.3, P);
    orc_sph_hankel1(11, 2.5, h);
    orc_cheb_nodes(8, t);
    orc_lagrange_basis(8, 0.1, ell);
    orc_lagrange_basis_deriv(8, 0.1, del);
    const int L = orc_gegenbauer_rank(20.0, 0.25, 1e-3);
    double *s = malloc(sizeof(double) * 3 * 2 * (size_t)L * (L + 1)), *w = malloc(sizeof(double) * 2 * (size_t)L * (L + 1));
    const int64_t nq = orc_sphere_quadrature(L, s, w);
    double *D = malloc(sizeof(double) * 2 * (size_t)nq);
    const double r0[3] = {0.5, 0.25, 0.0};
    orc_gegenbauer_diag(L, 20.0, r0, D);
    double *yb = malloc(sizeof(double) * 3 * 50), *ub = malloc(sizeof(double) * 2 * 50), *vb = calloc(100, sizeof(double));
    for (int i = 0; i < 150; ++i) yb[i] = 0.1 * (unif() - 0.5);
    input(ub, 50);
    double *ut = malloc(sizeof(double) * 2 * (size_t)nq);
    orc_grid_forward(32, 6, 13.8, 0.25 / 25.0, 20.0, L, yb, ub, 50, ut);
    orc_grid_backward(32, 6, 13.8, 0.25 / 25.0, 20.0, L, ut, yb, 50, vb);
    (void)orc_es_hat(6, 13.8, 1.0);
    double *T = malloc(sizeof(double) * 2 * 64 * 64), *A = malloc(sizeof(double) * 2 * 64 * 64),
           *B = malloc(sizeof(double) * 2 * 64 * 64);
    for (int i = 0; i < 64; ++i)
        for (int j = 0; j < 64; ++j) {
            T[2 * (64 * i + j)] = 1.0 / (1.0 + fabs((double)(i - j)) + 0.1 * i);
            T[2 * (64 * i + j) + 1] = 0.0;
        }
    const int rank = orc_aca(64, T, 1e-6, A, B);
    printf("aca rank %d, threads %d\n", rank, orc_num_threads());
    free(X);
    free(Y);
    free(N);
    free(Z);
    free(s);
    free(w);
    free(D);
    free(yb);
    free(ub);
    free(vb);
    free(ut);
    free(T);
    free(A);
    free(B);
    printf("failures %d\n", failures);
    return failures ? 1 : 0;
}
