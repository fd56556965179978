"""Pins of the oracle's adaptive cross approximation of the Lagrange transfer matrices (Sec. 2.2.2,
eq. ffmACAmatvec: T ~ A B^T, the product applied as A (B^T u~); reading R21: complete pivoting, stopping as
soon as |T - A B^T|_F <= tol |T|_F, tol = eps / 4 in the FFM).

The pins: matrices of known rank are reproduced to rounding with exactly that rank; on transfer matrices of
the Laplace and Helmholtz kernels the relative Frobenius error (computed here with numpy) is within the
tolerance, the rank is never below the optimal (singular value) rank for that error and one fewer term would
miss it; the whole FFM with ACA factors stays within eps of FP64 dense rows and close to the FFM with full
transfer matrices.
"""
import math

import numpy as np
import pytest

import oracle
import ffm_workloads as W


def _transfer_matrix(r1, off, kernel, k, dl=1.0):
    """T[(abc), (a'b'c')] = G(|o dl + (dl/2)(xi - xi')|) on the first-kind Chebyshev tensor grid (numpy)."""
    t = np.cos((2.0 * np.arange(1, r1 + 1) - 1.0) * math.pi / (2.0 * r1))
    g = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
    d = np.asarray(off, float)[None, None, :] * dl + 0.5 * dl * (g[:, None, :] - g[None, :, :])
    r = np.linalg.norm(d, axis=2)
    G = 1.0 / (4.0 * math.pi * r)
    return G * np.exp(1j * k * r) if kernel == 1 else G.astype(np.complex128)


def _svd_rank(T, tol):
    s = np.linalg.svd(T, compute_uv=False)
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]          # tail[k] = |sigma_{k..}|
    return int(np.argmax(tail <= tol * np.linalg.norm(s))) if np.any(tail <= tol * np.linalg.norm(s)) else len(s)


def test_exact_low_rank_is_recovered(orc):
    rng = np.random.default_rng(1)
    for rank in (1, 5, 12):
        X = rng.standard_normal((60, rank)) + 1j * rng.standard_normal((60, rank))
        Y = rng.standard_normal((60, rank)) + 1j * rng.standard_normal((60, rank))
        T = X @ Y.T
        A, B = oracle.aca(T, 1e-12)
        assert A.shape[1] == rank
        assert np.linalg.norm(T - A @ B.T) <= 1e-12 * np.linalg.norm(T)
    A, B = oracle.aca(np.zeros((8, 8)), 1e-6)
    assert A.shape[1] == 0


@pytest.mark.parametrize("kernel,k,off", [(0, 0.0, (2, 0, 0)), (0, 0.0, (3, -2, 1)), (1, 2.0, (2, 1, 0)),
                                          (1, 3.0, (2, 2, 2))])
@pytest.mark.parametrize("r1,tol", [(4, 2.5e-4), (6, 2.5e-5)])
def test_transfer_matrices_within_tolerance(orc, kernel, k, off, r1, tol):
    T = _transfer_matrix(r1, off, kernel, k)
    A, B = oracle.aca(T, tol)
    err = np.linalg.norm(T - A @ B.T) / np.linalg.norm(T)
    opt = _svd_rank(T, tol)
    print("r1 %d off %s kernel %d: rank %d (optimal %d of %d), error %.2e (tol %.1e)"
          % (r1, off, kernel, A.shape[1], opt, T.shape[0], err, tol))
    assert err <= tol * (1 + 1e-9)
    assert opt <= A.shape[1] < T.shape[0] // 2
    k = A.shape[1]
    assert np.linalg.norm(T - A[:, :k - 1] @ B[:, :k - 1].T) > tol * np.linalg.norm(T)     # greedy: no term spare
    if kernel == 0:
        assert np.abs(A.imag).max() == 0 and np.abs(B.imag).max() == 0     # a real kernel gives real factors


def test_pivots_ignore_rounding_differences(orc):
    """Entries equal up to rounding (the tensor grid's mirror symmetry) pick the same pivot: a matrix and its
    copy perturbed by an ulp give the same rank and factors to rounding."""
    T = _transfer_matrix(5, (2, 0, 0), 0, 0.0)
    T2 = T * (1 + 2.0 ** -52 * np.sign(np.sin(np.arange(T.size))).reshape(T.shape))
    A, B = oracle.aca(T, 2.5e-4)
    A2, B2 = oracle.aca(T2, 2.5e-4)
    assert A.shape == A2.shape
    assert np.linalg.norm(A @ B.T - A2 @ B2.T) <= 1e-12 * np.linalg.norm(T)


@pytest.mark.parametrize("kernel,k,eps", [(0, 0.0, 1e-4), (1, 9.0, 1e-3)])
def test_ffm_with_aca_factors(orc, kernel, k, eps):
    """The FFM with ACA factors at every Lagrange level: within eps of FP64 dense rows, and within eps / 2 of the
    FFM with full transfer matrices (tolerance eps / 4 per transfer)."""
    rng = np.random.default_rng(12)
    X = W.sphere_points(12000, rng)
    wu = ((rng.standard_normal(12000) + 1j * rng.standard_normal(12000)) / 12000).astype(np.complex128)
    full = oracle.Plan(X, X, kernel, k, eps)
    lag = [l for l in range(1, full.leaf + 1) if full.method(l) == 1]
    assert lag
    aca = oracle.Plan(X, X, kernel, k, eps, aca=lag, aca_tol=eps / 4)
    vf, va = full.apply(wu), aca.apply(wu)
    rows = np.arange(0, 12000, 31)
    d = oracle.dense_rows(X, X, wu, kernel, k, rows)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    ranks = {l: np.mean(list(aca.aca_ranks(l, eps / 4).values())) for l in lag}
    print("kernel %d eps %g: mean ranks %s; aca vs full %.2e, vs dense %.2e (full %.2e)"
          % (kernel, eps, ranks, rel(va, vf), rel(va[rows], d), rel(vf[rows], d)))
    assert 0 < rel(va, vf) <= eps / 2
    assert rel(va[rows], d) <= eps
