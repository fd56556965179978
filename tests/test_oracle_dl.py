"""Pins of the oracle's normal derivative at the sources, dG/dn_y (x, y) = n_y . grad_y G(x - y): the kernel of the
double-layer operator of Sec. 4.2.1 (eq. doubleLayer), the second of the kernel derivatives.

The FFM differentiates only its source side: the near field uses the derivative kernel, Lagrange levels the
derivatives of the anterpolation polynomials (chain factor 2 / d_l), Gegenbauer levels the factor -ik (s . n) of
each plane wave.  Pins: the dense rows equal central differences of the potential under a shift of the sources
along their normals; Gauss's law for the Laplace double layer of a closed surface (-1 inside, 0 outside, with
G = 1 / (4 pi r) and area weights); the Helmholtz double layer of a uniform sphere from the n = 0 term of the
addition theorem; the transpose relation with the target-side derivative, densely and, to rounding, through the
two FFMs; the FFM within eps of dense rows, also through the grid form (-ik sum_c s_c times the source transforms
of u n_c).
"""
import math

import numpy as np
import pytest

import oracle
import ffm_workloads as W


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 6.5)])
def test_dense_rows_are_the_derivative_along_source_normals(orc, kernel, k):
    """(phi(Y + h N) - phi(Y - h N)) / 2h with phi the single-layer rows, error O(h^2)."""
    rng = np.random.default_rng(6)
    Y = W.sphere_points(400, rng)
    N = W.sphere_points(400, rng)
    X = W.sphere_points(30, rng) * 1.7
    wu = rng.standard_normal(400) + 1j * rng.standard_normal(400)
    rows = np.arange(30)
    got = oracle.dense_rows_dl(X, Y, wu, kernel, k, N, rows)
    errs = []
    for h in (1e-3, 5e-4):
        fd = (orc.dense_rows(X, Y + h * N, wu, kernel, k, rows) - orc.dense_rows(X, Y - h * N, wu, kernel, k, rows))
        errs.append(np.abs(fd / (2 * h) - got).max() / np.abs(got).max())
    assert errs[0] < 1e-5 and 3.0 < errs[0] / errs[1] < 5.0        # second order in h


@pytest.mark.parametrize("rho", [0.0, 0.3, 0.7, 1.6, 3.0])
def test_laplace_gauss_law(orc, rho):
    """sum_j n_j . grad_y G(x - y_j) w_j over an area quadrature of the unit sphere (outward normals) is -1 for x
    inside and 0 outside, wherever x is."""
    Y, w = W.shell_grid(64, 128)
    rng = np.random.default_rng(9)
    T = W.sphere_points(12, rng) * rho
    v = oracle.dense_rows_dl(T, Y, w.astype(np.complex128), 0, 0.0, Y, np.arange(12))
    ref = -1.0 if rho < 1 else 0.0
    assert np.abs(v - ref).max() < 1e-9


def _h0(z):
    return np.exp(1j * z) / (1j * z)


def _h0p(z):
    return np.exp(1j * z) * (1.0 / z + 1j / z ** 2)


def _j0(z):
    return math.sin(z) / z


def _j0p(z):
    return math.cos(z) / z - math.sin(z) / z ** 2


@pytest.mark.parametrize("k", [0.9, 3.7, 12.25])
@pytest.mark.parametrize("rho", [0.4, 2.0])
def test_helmholtz_shell_double_layer(orc, k, rho):
    """With G = e^{ikr} / (4 pi r), the integral of G(x - a y) dS(y) over the unit sphere is ik j0(k r<) h0(k r>)
    (r< and r> the smaller and the larger of a and |x|); its derivative in a at a = 1 gives
    i k^2 j0(k rho) h0'(k) inside and i k^2 h0(k rho) j0'(k) outside."""
    Y, w = W.shell_grid(64, 128)
    rng = np.random.default_rng(4)
    T = W.sphere_points(20, rng) * rho
    v = oracle.dense_rows_dl(T, Y, w.astype(np.complex128), 1, k, Y, np.arange(20))
    if rho < 1:
        ref = 1j * k * k * _j0(k * rho) * _h0p(k)
    else:
        ref = 1j * k * k * _h0(k * rho) * _j0p(k)
    assert np.abs(v - ref).max() < 1e-9 * max(1.0, abs(ref))


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 5.0)])
def test_dense_transpose_of_target_derivative(orc, kernel, k):
    """dG/dn_y (x_i, y_j) = dG/dn_x (y_j, x_i) with the same normal n_j: the double-layer matrix is the plain
    transpose of the target-side derivative matrix with targets and sources exchanged."""
    rng = np.random.default_rng(12)
    X = W.sphere_points(150, rng) * 0.8
    Y = W.sphere_points(170, rng)
    N = W.sphere_points(170, rng)
    u = rng.standard_normal(150) + 1j * rng.standard_normal(150)
    wv = rng.standard_normal(170) + 1j * rng.standard_normal(170)
    a = np.dot(u, oracle.dense_rows_dl(X, Y, wv, kernel, k, N, np.arange(150)))
    b = np.dot(wv, oracle.dense_rows_dn(Y, X, u, kernel, k, N, np.arange(170)))
    assert abs(a - b) < 1e-12 * abs(a)


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 9.0), (1, 30.0)])
def test_ffm_double_layer_within_eps(orc, kernel, k):
    """The whole FFM of the double-layer kernel (sources on the unit sphere with their outward normals, targets on
    a second sphere): within eps of FP64 dense rows, at Lagrange and Gegenbauer levels, and more accurate at
    smaller eps; and the transpose relation with the target-side FFM holds to the same eps."""
    rng = np.random.default_rng(22)
    Y = W.sphere_points(6000, rng)
    X = W.sphere_points(5000, rng) * 0.98
    wu = (rng.standard_normal(6000) + 1j * rng.standard_normal(6000)) / 6000
    rows = np.arange(0, 5000, 11)
    d = oracle.dense_rows_dl(X, Y, wu, kernel, k, Y, rows)
    errs, prod = [], {}
    for eps in (1e-3, 1e-5):
        p = oracle.Plan(X, Y, kernel + 4, k, eps, n_leaf=32, source_normals=Y)
        meth = [p.method(l) for l in range(1, p.leaf + 1)]
        prod[eps] = v = p.apply(wu)
        errs.append(float(np.linalg.norm(v[rows] - d) / np.linalg.norm(d)))
        print("kernel %d k %g eps %g: methods %s, error %.2e" % (kernel, k, eps, meth, errs[-1]))
        assert errs[-1] <= eps
    assert errs[1] < errs[0]
    # <u, DL w> = <w, DN u> through the two FFMs at eps 1e-3 (the DN plan takes the sources as targets with the
    # same normals).  It holds to rounding, not only to eps: with the sets exchanged the two plans have the same
    # boxes and lists, each source-side step of one is the transpose of the target-side step of the other, and the
    # transfer kernels are symmetric under exchanging the centres.
    u = (rng.standard_normal(5000) + 1j * rng.standard_normal(5000)) / 5000
    q = oracle.Plan(Y, X, kernel + 2, k, 1e-3, n_leaf=32, normals=Y)
    a = np.dot(u, prod[1e-3])
    b = np.dot(wu, q.apply(u))
    scale = np.linalg.norm(u) * np.linalg.norm(prod[1e-3])
    print("transpose relation: %.2e of |u| |DL w|" % (abs(a - b) / scale))
    assert abs(a - b) < 1e-12 * scale


def test_ffm_double_layer_grid_form(orc):
    """The double layer through the grid form (level 2): -ik sum_c s_c (the grid form's source transforms of the
    densities u n_c), within eps of dense rows and of the direct form."""
    rng = np.random.default_rng(27)
    Y = W.sphere_points(4000, rng)
    X = W.sphere_points(3000, rng) * 0.98
    wu = (rng.standard_normal(4000) + 1j * rng.standard_normal(4000)) / 4000
    rows = np.arange(0, 3000, 7)
    d = oracle.dense_rows_dl(X, Y, wu, 1, 30.0, Y, rows)
    direct = oracle.Plan(X, Y, 5, 30.0, 1e-3, n_leaf=32, source_normals=Y)
    assert direct.method(2) == 2
    g = oracle.Plan(X, Y, 5, 30.0, 1e-3, n_leaf=32, source_normals=Y, grid={2: (32, 6, 2.3 * 6)})
    vg, vd = g.apply(wu), direct.apply(wu)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print("grid form %.2e, direct %.2e, grid against direct %.2e" % (rel(vg[rows], d), rel(vd[rows], d), rel(vg, vd)))
    assert rel(vg[rows], d) <= 1e-3 and rel(vd[rows], d) <= 1e-3 and rel(vg, vd) <= 1e-3
    assert rel(vg, vd) > 1e-12          # the grid form did run
