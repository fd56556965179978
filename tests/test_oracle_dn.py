"""Pins of the oracle's normal derivative at the targets, dG/dn_x (x, y) = n_x . grad_x G(x - y): the kernel of
the adjoint double-layer operator of Sec. 4.2.1 (eq. doubleLayer), the first of the kernel derivatives.

The FFM differentiates only its target side: the near field uses the derivative kernel, Lagrange levels the
derivatives of the interpolation polynomials (chain factor 2 / d_l), Gegenbauer levels the factor ik (s . n) of
each plane wave.  Pins: the polynomial derivatives reproduce those of polynomials of degree < r1; the dense
rows equal central differences of the potential along n; the radial derivative of a uniform shell's potential
(closed forms from the n = 0 term of the addition theorem) inside and outside; the FFM within eps of dense rows,
also through the grid form (n . the target transforms of ik s_c v~).
"""
import math

import numpy as np
import pytest

import oracle
import ffm_workloads as W


@pytest.mark.parametrize("r1", [3, 5, 8])
def test_basis_derivatives_reproduce_polynomial_derivatives(orc, r1):
    rng = np.random.default_rng(r1)
    nodes = orc.cheb_nodes(r1)
    for deg in range(r1):
        c = rng.standard_normal(deg + 1)
        dc = np.polyder(c) if deg > 0 else np.zeros(1)
        for t in np.linspace(-1, 1, 7):
            d = oracle.lagrange_basis_deriv(r1, t)
            assert abs(np.dot(d, np.polyval(c, nodes)) - np.polyval(dc, t)) < 1e-11 * max(1.0, np.abs(c).sum())
        assert abs(oracle.lagrange_basis_deriv(r1, 0.3).sum()) < 1e-12      # derivative of the partition of unity


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 6.5)])
def test_dense_rows_are_the_derivative_along_n(orc, kernel, k):
    """Central differences of the potential at x +- h n, with error O(h^2)."""
    rng = np.random.default_rng(5)
    Y = W.sphere_points(400, rng)
    X = W.sphere_points(30, rng) * 1.7
    N = W.sphere_points(30, rng)
    wu = rng.standard_normal(400) + 1j * rng.standard_normal(400)
    rows = np.arange(30)
    got = oracle.dense_rows_dn(X, Y, wu, kernel, k, N, rows)
    errs = []
    for h in (1e-3, 5e-4):
        fd = (orc.dense_rows(X + h * N, Y, wu, kernel, k, rows) - orc.dense_rows(X - h * N, Y, wu, kernel, k, rows))
        errs.append(np.abs(fd / (2 * h) - got).max() / np.abs(got).max())
    assert errs[0] < 1e-5 and 3.0 < errs[0] / errs[1] < 5.0        # second order in h


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 3.7), (1, 12.25)])
@pytest.mark.parametrize("rho", [0.5, 2.0])
def test_dense_shell_radial_derivative(orc, kernel, k, rho):
    """d/d rho of the uniform shell's potential: inside Laplace 0, Helmholtz e^{ik} d/d rho [sin(k rho)/(k rho)];
    outside Laplace -1/rho^2, Helmholtz sin(k) d/d rho [e^{ik rho}/(k rho)]."""
    Y, w = W.shell_grid(48, 96)
    rng = np.random.default_rng(3)
    Nrm = W.sphere_points(20, rng)
    T = Nrm * rho
    v = oracle.dense_rows_dn(T, Y, w.astype(np.complex128), kernel, k, Nrm, np.arange(20))
    if kernel == 0:
        ref = 0.0 if rho < 1 else -1.0 / rho ** 2
    elif rho < 1:
        x = k * rho
        ref = np.exp(1j * k) * k * (math.cos(x) / x - math.sin(x) / x ** 2)
    else:
        ref = math.sin(k) * (1j * k * np.exp(1j * k * rho) / (k * rho) - np.exp(1j * k * rho) / (k * rho ** 2))
    assert np.abs(v - ref).max() < 1e-9


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 9.0), (1, 30.0)])
def test_ffm_normal_derivative_within_eps(orc, kernel, k):
    """The whole FFM of the normal-derivative kernel (targets on a second sphere, their radial normals; sources on
    the unit sphere): within eps of FP64 dense rows, at Lagrange and Gegenbauer levels, and more accurate at
    smaller eps."""
    rng = np.random.default_rng(21)
    Y = W.sphere_points(6000, rng)
    N = W.sphere_points(5000, rng)
    X = N * 0.98
    wu = (rng.standard_normal(6000) + 1j * rng.standard_normal(6000)) / 6000
    rows = np.arange(0, 5000, 11)
    d = oracle.dense_rows_dn(X, Y, wu, kernel, k, N, rows)
    errs = []
    for eps in (1e-3, 1e-5):
        p = oracle.Plan(X, Y, kernel + 2, k, eps, n_leaf=32, normals=N)
        meth = [p.method(l) for l in range(1, p.leaf + 1)]
        v = p.apply(wu)
        errs.append(float(np.linalg.norm(v[rows] - d) / np.linalg.norm(d)))
        print("kernel %d k %g eps %g: methods %s, error %.2e" % (kernel, k, eps, meth, errs[-1]))
        assert errs[-1] <= eps
    assert errs[1] < errs[0]


def test_ffm_normal_derivative_grid_form(orc):
    """The normal derivative at the targets through the grid form (level 2): n . (the grid form's target
    transforms of ik s_c v~), within eps of dense rows and of the direct form."""
    rng = np.random.default_rng(26)
    Y = W.sphere_points(4000, rng)
    N = W.sphere_points(3000, rng)
    X = N * 0.98
    wu = (rng.standard_normal(4000) + 1j * rng.standard_normal(4000)) / 4000
    rows = np.arange(0, 3000, 7)
    d = oracle.dense_rows_dn(X, Y, wu, 1, 30.0, N, rows)
    direct = oracle.Plan(X, Y, 3, 30.0, 1e-3, n_leaf=32, normals=N)
    assert direct.method(2) == 2
    g = oracle.Plan(X, Y, 3, 30.0, 1e-3, n_leaf=32, normals=N, grid={2: (32, 6, 2.3 * 6)})
    vg, vd = g.apply(wu), direct.apply(wu)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print("grid form %.2e, direct %.2e, grid against direct %.2e" % (rel(vg[rows], d), rel(vd[rows], d), rel(vg, vd)))
    assert rel(vg[rows], d) <= 1e-3 and rel(vd[rows], d) <= 1e-3 and rel(vg, vd) <= 1e-3
    assert rel(vg, vd) > 1e-12          # the grid form did run
