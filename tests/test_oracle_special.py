"""Pins of the oracle's building blocks against independent libraries and closed forms.

Paper: Sec. 2.2.2 (Chebyshev/Lagrange interpolation), Sec. 2.2.3 (Gegenbauer series,
spherical quadrature, eqs. gegenbauerIntegral..gegenbauerQuadrature), Sec. 3.3 (n_Q = 2L(L+1)).
"""
import math

import numpy as np
import pytest
import scipy.special as sp


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 65, 165, 400])
def test_gauss_legendre_matches_numpy(orc, n):
    x, w = orc.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    o = np.argsort(x)
    assert np.allclose(x[o], xr, atol=1e-14, rtol=0)
    # numpy's own weights drift by ~1e-14 at large n; exactness below is the sharper pin
    assert np.allclose(w[o], wr, atol=5e-14, rtol=1e-9)
    # exact for polynomials of degree <= 2n - 1
    for j in range(0, 2 * n, max(1, n // 4)):
        exact = 2.0 / (j + 1) if j % 2 == 0 else 0.0
        assert abs(np.dot(w, x ** j) - exact) < 1e-13


@pytest.mark.parametrize("t", [-1.0, -0.73, 0.0, 0.1234, 0.999])
def test_legendre_matches_scipy(orc, t):
    P = orc.legendre_p(60, t)
    ref = sp.eval_legendre(np.arange(61), t)
    assert np.allclose(P, ref, atol=1e-13, rtol=1e-12)


@pytest.mark.parametrize("z", [0.7, 3.0, 11.34, 45.4, 181.5])
def test_spherical_hankel_matches_scipy(orc, z):
    L = int(z * 1.5 + 20)
    h = orc.sph_hankel1(L, z)
    p = np.arange(L + 1)
    ref = sp.spherical_jn(p, z) + 1j * sp.spherical_yn(p, z)
    # the y_p part dominates above the turning point; compare relative to |h_p|
    rel = np.abs(h - ref) / np.abs(ref)
    assert rel.max() < 1e-9, rel.max()


def test_hankel_closed_forms(orc):
    z = 2.5
    h = orc.sph_hankel1(2, z)
    e = np.exp(1j * z)
    assert abs(h[0] - (-1j * e / z)) < 1e-15
    assert abs(h[1] - (-e * (z + 1j) / z ** 2)) < 1e-15
    # h_2 = i e^{iz} (z^2 + 3iz - 3) / z^3
    assert abs(h[2] - (1j * e * (z * z + 3j * z - 3) / z ** 3)) < 1e-14


@pytest.mark.parametrize("r1", [1, 2, 4, 6, 9])
def test_chebyshev_nodes_first_kind(orc, r1):
    t = np.sort(orc.cheb_nodes(r1))
    ref = np.sort(np.polynomial.chebyshev.chebpts1(r1))
    assert np.allclose(t, ref, atol=1e-15)
    # nodes of the first kind are the zeros of T_{r1}
    assert np.allclose(np.cos(r1 * np.arccos(t)), 0.0, atol=1e-13)


@pytest.mark.parametrize("r1", [2, 4, 6, 8])
def test_lagrange_reproduces_polynomials(orc, r1):
    rng = np.random.default_rng(11)
    nodes = orc.cheb_nodes(r1)
    for deg in range(r1):
        c = rng.standard_normal(deg + 1)
        for t in np.linspace(-1, 1, 9):
            ell = orc.lagrange_basis(r1, t)
            assert abs(ell.sum() - 1.0) < 1e-13          # partition of unity
            interp = np.dot(ell, np.polyval(c, nodes))
            assert abs(interp - np.polyval(c, t)) < 1e-12 * max(1.0, np.abs(c).sum())
    # a polynomial of degree r1 is NOT reproduced (the interpolant is not trivial)
    ell = orc.lagrange_basis(r1, 0.3)
    assert abs(np.dot(ell, nodes ** r1) - 0.3 ** r1) > 1e-6


@pytest.mark.parametrize("kdl", [5.67, 11.3])
def test_gegenbauer_rank_meets_eps_at_the_closest_offset(orc, kdl):
    """The rank of eq. (gegenbauerRank) read with the natural log (reading R7) keeps the single-pair error of the
    expansion below eps = 1e-3 for every sampled pair of points at the closest admissible offset (2, 0, 0), the
    worst case of a level; the decimal-log reading, 4 orders fewer, fails it at the leaf-like level kd = 5.67.
    Pinned against e^{ikr} / (4 pi r) itself, not against the formula."""
    k, eps = 181.499, 1e-3
    d = kdl / k

    def worst(L):
        s, _ = orc.sphere_quadrature(L)
        r0 = np.array([2.0, 0.0, 0.0]) * d
        D = orc.gegenbauer_diag(L, k, r0)
        rng = np.random.default_rng(7)
        xs = (rng.random((60, 3)) - 0.5) * d
        ys = (rng.random((60, 3)) - 0.5) * d
        e = 0.0
        for x, y in zip(xs, ys):
            r = np.linalg.norm(r0 + x - y)
            exact = np.exp(1j * k * r) / (4 * math.pi * r)
            approx = np.sum(np.exp(1j * k * (s @ x)) * D * np.exp(-1j * k * (s @ y)))
            e = max(e, abs(approx - exact) / abs(exact))
        return e

    L = orc.gegenbauer_rank(k, d, eps)
    assert worst(L) < eps
    if kdl < 6:
        assert worst(int(math.floor(k * math.sqrt(3) * d - math.log10(eps)))) > eps
    # the rank grows with the box: one more level up needs more terms
    assert orc.gegenbauer_rank(k, 2 * d, eps) > L
    assert orc.gegenbauer_rank(0.0, 1.0, 0.9) == 1          # L >= 1


@pytest.mark.parametrize("L", [1, 2, 5, 16, 40])
def test_sphere_quadrature_exactness(orc, L):
    s, w = orc.sphere_quadrature(L)
    assert s.shape[0] == 2 * L * (L + 1)
    assert abs(w.sum() - 4 * math.pi) < 1e-12
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-14)
    # int_{S^2} P_p(s.a) ds = 4 pi delta_{p0}, exact for p <= 2L - 1 (any unit a)
    rng = np.random.default_rng(L)
    a = rng.standard_normal(3)
    a /= np.linalg.norm(a)
    t = s @ a
    for p in range(0, 2 * L):
        val = np.dot(w, sp.eval_legendre(p, t))
        assert abs(val - (4 * math.pi if p == 0 else 0.0)) < 1e-11, (p, val)
    # antipodal symmetry: -s is a node with the same weight
    S = {tuple(np.round(x, 12)) for x in s}
    assert all(tuple(np.round(-x, 12)) in S for x in s)


@pytest.mark.parametrize("kdl,off", [(5.67, (2, 0, 0)), (5.67, (3, -2, 1)), (11.3, (2, 2, 2)),
                                     (45.4, (2, 1, 0)), (90.7, (3, 0, -1))])
def test_gegenbauer_single_pair_identity(orc, kdl, off):
    """e^{ikr}/(4 pi r) ~ sum_q e^{ik s_q.(x-x0)} D(q) e^{-ik s_q.(y-y0)} for admissible boxes."""
    k = 181.499
    d = kdl / k
    eps = 1e-3
    L = orc.gegenbauer_rank(k, d, eps)
    s, _ = orc.sphere_quadrature(L)
    r0 = np.array(off, dtype=float) * d
    D = orc.gegenbauer_diag(L, k, r0)
    rng = np.random.default_rng(7)
    xs = (rng.random((40, 3)) - 0.5) * d
    ys = (rng.random((40, 3)) - 0.5) * d
    rel = []
    for x, y in zip(xs, ys):
        r = np.linalg.norm(r0 + x - y)
        exact = np.exp(1j * k * r) / (4 * math.pi * r)
        approx = np.sum(np.exp(1j * k * (s @ x)) * D * np.exp(-1j * k * (s @ y)))
        rel.append(abs(approx - exact) / abs(exact))
    rel = np.array(rel)
    assert np.median(rel) < eps, np.median(rel)
    assert rel.max() < 10 * eps, rel.max()


def test_gegenbauer_needs_monopole_term(orc):
    """Dropping the p = 0 term of the series (as printed, p starting at 1) fails grossly."""
    k, d = 181.499, 0.03125
    L = orc.gegenbauer_rank(k, d, 1e-3)
    s, w = orc.sphere_quadrature(L)
    r0 = np.array([2.0, 0.0, 0.0]) * d
    D = orc.gegenbauer_diag(L, k, r0)
    rn = np.linalg.norm(r0)
    h0 = orc.sph_hankel1(0, k * rn)[0]
    D_no0 = D - (1j * k / (4 * math.pi)) * w * (h0 / (4 * math.pi))
    x = np.array([0.01, -0.003, 0.004])
    y = np.array([-0.002, 0.005, 0.001])
    r = np.linalg.norm(r0 + x - y)
    exact = np.exp(1j * k * r) / (4 * math.pi * r)
    good = np.sum(np.exp(1j * k * (s @ x)) * D * np.exp(-1j * k * (s @ y)))
    bad = np.sum(np.exp(1j * k * (s @ x)) * D_no0 * np.exp(-1j * k * (s @ y)))
    assert abs(good - exact) / abs(exact) < 1e-3
    assert abs(bad - exact) / abs(exact) > 0.1
