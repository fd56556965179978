"""Pins of the oracle's grid form of the plane-wave transforms (readings R16-R18; the fast evaluation of the
transforms asked for in the remark closing Sec. 2.2.3).

The grid form approximates e^{-ik s.(y - c)} along each axis by Poisson summation: spreading a point onto the
grid with the kernel phi and summing the grid against the plane wave gives e^{-i om y} phihat(om h) plus the
aliased terms phihat(om h + 2 pi m), m != 0.  So for one point and one direction the relative error of the
whole transform is at most prod_d (1 + B_d) - 1, with B_d = sum_{m != 0} |phihat(om_d h + 2 pi m)| / phihat(om_d h).
These tests evaluate phihat independently (scipy's adaptive quadrature in the original variable) and check the
oracle against the exact plane waves within that bound, and its kernel transform against scipy.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle


def _es(t, w, beta):
    x = 2.0 * t / w
    return np.exp(beta * (np.sqrt(np.maximum(0.0, 1.0 - x * x)) - 1.0)) * (np.abs(x) < 1.0)


def _phihat(w, beta, xi):
    f = lambda t: _es(t, w, beta) * math.cos(xi * t)
    val, _ = integrate.quad(f, -0.5 * w, 0.5 * w, limit=200, epsabs=1e-14, epsrel=1e-12)
    return val


def _alias(w, beta, om):
    """One-axis aliasing ratio at frequency om (node units), terms |m| <= 4."""
    s = sum(abs(_phihat(w, beta, om + 2 * math.pi * m)) for m in range(-4, 5) if m != 0)
    return s / _phihat(w, beta, om)


@pytest.mark.parametrize("w,beta,xi", [(4, 8.8, 0.0), (5, 11.0, 1.3), (6, 13.8, 2.09), (8, 18.4, 0.7),
                                       (6, 13.8, 2 * math.pi + 1.0)])
def test_kernel_transform_matches_scipy(orc, w, beta, xi):
    assert abs(oracle.es_hat(w, beta, xi) - _phihat(w, beta, xi)) <= 1e-11 * _phihat(w, beta, 0.0)


@pytest.mark.parametrize("p,w,c,k,L", [(16, 5, 2.2, 25.0, 12), (32, 6, 2.3, 60.0, 20), (32, 4, 2.0, 45.0, 16)])
def test_forward_single_points_within_aliasing_bound(orc, p, w, c, k, L):
    """Each point alone: u~(q) against the exact plane wave e^{-ik s_q.y}, for every direction, within
    prod_d (1 + B_d(q)) - 1 (B from scipy); the bound is checked on a sample of directions, the maximum
    deviation over all directions against the largest sampled bound times 1.5."""
    rng = np.random.default_rng(p + w)
    beta = c * w
    dl = 0.5
    h = dl / (p - 1 - w)
    assert k * h <= math.pi / 1.5 + 1e-9
    s, _ = oracle.sphere_quadrature(L)
    qs = rng.choice(s.shape[0], 12, replace=False)
    bound = np.array([np.prod([1.0 + _alias(w, beta, k * s[q, d] * h) for d in range(3)]) - 1.0 for q in qs])
    for _ in range(3):
        y = (rng.random((1, 3)) - 0.5) * dl
        ut = oracle.grid_forward(p, w, beta, h, k, L, y, np.array([1.0 + 0.0j]))
        exact = np.exp(-1j * k * (s @ y[0]))
        err = np.abs(ut - exact)
        assert np.all(err[qs] <= bound * (1 + 1e-6) + 1e-13), (err[qs], bound)
        assert err.max() <= 1.5 * bound.max()
        assert err.max() > 1e-12            # the grid form is an approximation, not the direct sum


def test_backward_single_target_within_aliasing_bound(orc):
    """sum_q e^{ik s_q.x} vt(q) at one point, grid against direct, within sum_q |vt(q)| (prod_d (1 + B_d) - 1)."""
    rng = np.random.default_rng(3)
    p, w, beta, k, L, dl = 32, 6, 13.8, 50.0, 18, 0.5
    h = dl / (p - 1 - w)
    s, _ = oracle.sphere_quadrature(L)
    worst = max(np.prod([1.0 + _alias(w, beta, k * abs(s[q, d]) * h) for d in range(3)]) - 1.0
                for q in range(0, s.shape[0], 7))
    vt = rng.standard_normal(s.shape[0]) + 1j * rng.standard_normal(s.shape[0])
    x = (rng.random((5, 3)) - 0.5) * dl
    got = oracle.grid_backward(p, w, beta, h, k, L, vt, x)
    direct = np.exp(1j * k * (x @ s.T)) @ vt
    assert np.all(np.abs(got - direct) <= 1.5 * worst * np.abs(vt).sum())
    # a plausible slip, conjugating the target phases, would be far outside the bound
    wrong = np.exp(-1j * k * (x @ s.T)) @ vt
    assert np.all(np.abs(wrong - direct) > 10 * 1.5 * worst * np.abs(vt).sum())


def test_forward_is_linear_and_sums_boxes(orc):
    """Spreading is linear: the transform of many points equals the sum of their single-point transforms."""
    rng = np.random.default_rng(5)
    p, w, beta, k, L, dl = 16, 5, 11.0, 20.0, 10, 0.5
    h = dl / (p - 1 - w)
    y = (rng.random((40, 3)) - 0.5) * dl
    u = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    whole = oracle.grid_forward(p, w, beta, h, k, L, y, u)
    parts = sum(oracle.grid_forward(p, w, beta, h, k, L, y[j:j + 1], u[j:j + 1]) for j in range(40))
    assert np.allclose(whole, parts, rtol=0, atol=1e-12 * np.abs(whole).max())


def test_grid_ffm_against_direct_and_dense(orc):
    """The whole FFM with grid-form transforms at every Gegenbauer level: within eps of FP64 dense rows, and
    within 2 E of the direct-sum FFM, E = max over directions of prod_d (1 + B_d) - 1 (one transform on each
    side of the transfer)."""
    import ffm_workloads as W
    w_ = W.helmholtz_sphere(6000, seed=11, k=40.0, n_rows=256)
    op_d = oracle.Plan(w_.X, w_.X, 1, w_.k, w_.eps, n_leaf=32)
    grid, Emax = {}, 0.0
    for l in range(1, op_d.leaf + 1):
        if op_d.method(l) != 2:
            continue
        dl = op_d.d0 * 2.0 ** -l
        gw, beta = 6, 13.8
        p = 16 * math.ceil((dl * w_.k / (math.pi / 1.5) + 1 + gw) / 16)    # k h <= pi / 1.5
        h = dl / (p - 1 - gw)
        assert w_.k * h <= math.pi / 1.5
        grid[l] = (p, gw, beta)
        B = _alias(gw, beta, w_.k * h)
        Emax = max(Emax, (1 + B) ** 3 - 1)
    assert grid
    op_g = oracle.Plan(w_.X, w_.X, 1, w_.k, w_.eps, n_leaf=32, grid=grid)
    vd = op_d.apply(w_.wu)
    vg = op_g.apply(w_.wu)
    dense = oracle.dense_rows(w_.X, w_.X, w_.wu, 1, w_.k, w_.rows)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    print("grid levels %s: grid vs direct %.2e (bound %.2e), vs dense %.2e (direct %.2e)"
          % (grid, rel(vg, vd), 2 * Emax, rel(vg[w_.rows], dense), rel(vd[w_.rows], dense)))
    assert 0 < rel(vg, vd) <= 2 * Emax
    assert rel(vg[w_.rows], dense) <= w_.eps
