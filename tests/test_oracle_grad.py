"""Pins of the oracle's gradient at the targets, grad_x G(x - y): three components per target, the vector kernel
that the integral operators of Sec. 4.2.2 (the MFIE's n x curl of the single layer) are built from.

The oracle takes component c as the normal derivative at the targets with n = e_c (the target-side derivative of
the FFM, pinned in test_oracle_dn.py).  Pins: the dense rows equal central differences of the potential along
each axis; the gradient of a uniform shell's potential (radial, closed forms from the n = 0 term of the addition
theorem) inside and outside; the FFM's components combine into the normal-derivative FFM for any normals, to
rounding; the FFM within eps of dense rows at Lagrange and Gegenbauer levels.
"""
import math

import numpy as np
import pytest

import oracle
import ffm_workloads as W


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 6.5)])
def test_dense_rows_are_central_differences(orc, kernel, k):
    rng = np.random.default_rng(15)
    Y = W.sphere_points(400, rng)
    X = W.sphere_points(30, rng) * 1.6
    wu = rng.standard_normal(400) + 1j * rng.standard_normal(400)
    rows = np.arange(30)
    got = oracle.dense_rows_grad(X, Y, wu, kernel, k, rows)
    assert got.shape == (30, 3)
    for c in range(3):
        e = np.zeros(3)
        e[c] = 1.0
        errs = []
        for h in (1e-3, 5e-4):
            fd = orc.dense_rows(X + h * e, Y, wu, kernel, k, rows) - orc.dense_rows(X - h * e, Y, wu, kernel, k, rows)
            errs.append(np.abs(fd / (2 * h) - got[:, c]).max() / np.abs(got).max())
        assert errs[0] < 1e-5 and 3.0 < errs[0] / errs[1] < 5.0        # second order in h


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 3.7), (1, 12.25)])
@pytest.mark.parametrize("rho", [0.5, 2.0])
def test_dense_shell_gradient(orc, kernel, k, rho):
    """The uniform shell's potential depends on |x| alone, so its gradient is x / |x| times the radial derivative:
    inside Laplace 0, Helmholtz e^{ik} d/d rho [sin(k rho)/(k rho)]; outside Laplace -1/rho^2, Helmholtz
    sin(k) d/d rho [e^{ik rho}/(k rho)]."""
    Y, w = W.shell_grid(48, 96)
    rng = np.random.default_rng(5)
    D = W.sphere_points(20, rng)
    v = oracle.dense_rows_grad(D * rho, Y, w.astype(np.complex128), kernel, k, np.arange(20))
    if kernel == 0:
        dr = 0.0 if rho < 1 else -1.0 / rho ** 2
    elif rho < 1:
        x = k * rho
        dr = np.exp(1j * k) * k * (math.cos(x) / x - math.sin(x) / x ** 2)
    else:
        dr = math.sin(k) * (1j * k * np.exp(1j * k * rho) / (k * rho) - np.exp(1j * k * rho) / (k * rho ** 2))
    assert np.abs(v - D * dr).max() < 1e-9


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 9.0), (1, 30.0)])
def test_ffm_gradient_within_eps(orc, kernel, k):
    """The whole FFM of the gradient (targets on a second sphere): within eps of FP64 dense rows at Lagrange and
    Gegenbauer levels, more accurate at smaller eps; n . (its components) is the normal-derivative FFM with
    target normals n, to rounding."""
    rng = np.random.default_rng(23)
    Y = W.sphere_points(6000, rng)
    N = W.sphere_points(5000, rng)
    X = N * 0.98
    wu = (rng.standard_normal(6000) + 1j * rng.standard_normal(6000)) / 6000
    rows = np.arange(0, 5000, 11)
    d = oracle.dense_rows_grad(X, Y, wu, kernel, k, rows)
    errs, prod = [], {}
    for eps in (1e-3, 1e-4):
        p = oracle.Plan(X, Y, kernel + 6, k, eps, n_leaf=32)
        meth = [p.method(l) for l in range(1, p.leaf + 1)]
        prod[eps] = v = p.apply(wu)
        assert v.shape == (5000, 3)
        errs.append(float(np.linalg.norm(v[rows] - d) / np.linalg.norm(d)))
        print("kernel %d k %g eps %g: methods %s, error %.2e" % (kernel, k, eps, meth, errs[-1]))
        assert errs[-1] <= eps
    assert errs[1] < errs[0]
    dn = oracle.Plan(X, Y, kernel + 2, k, 1e-3, n_leaf=32, normals=N).apply(wu)
    comb = (prod[1e-3] * N).sum(axis=1)
    print("n . grad against the normal-derivative product: %.2e" % (np.linalg.norm(comb - dn) / np.linalg.norm(dn)))
    assert np.linalg.norm(comb - dn) <= 1e-12 * np.linalg.norm(dn)


def test_ffm_gradient_grid_form(orc):
    """The gradient through the grid form of the plane-wave transforms (level 2): component c is the grid form's
    target transform of ik s_c v~, within eps of dense rows and of the direct form."""
    rng = np.random.default_rng(24)
    Y = W.sphere_points(4000, rng)
    X = W.sphere_points(3000, rng) * 0.98
    wu = (rng.standard_normal(4000) + 1j * rng.standard_normal(4000)) / 4000
    rows = np.arange(0, 3000, 7)
    d = oracle.dense_rows_grad(X, Y, wu, 1, 30.0, rows)
    direct = oracle.Plan(X, Y, 7, 30.0, 1e-3, n_leaf=32)
    assert direct.method(2) == 2
    g = oracle.Plan(X, Y, 7, 30.0, 1e-3, n_leaf=32, grid={2: (32, 6, 2.3 * 6)})
    vg, vd = g.apply(wu), direct.apply(wu)
    eg, ed = rel_err(vg[rows], d), rel_err(vd[rows], d)
    print("grid form %.2e, direct %.2e, grid against direct %.2e" % (eg, ed, rel_err(vg, vd)))
    assert eg <= 1e-3 and ed <= 1e-3 and rel_err(vg, vd) <= 1e-3
    assert rel_err(vg, vd) > 1e-12          # the grid form did run


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
