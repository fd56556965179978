"""FP64 oracle of the single-layer boundary-integral equation on a sphere (paper Sec. 4.2), dense.

TEST INFRASTRUCTURE.  Only ``tests/`` may import this module.  It shares no code with the GPU library and
never imports it.  Plain numpy in FP64; the dense Green sums go through the oracle's C library.

The discrete operator is the Nystrom matrix on quadrature nodes x_j with weights w_j,

    A_ij = G(x_i, x_j) w_j  (i != j),     A_ii = lambda_0 - sum_{j != i} G(x_i, x_j) w_j,

i.e. the punctured quadrature of the single-layer integral plus singularity subtraction against the constant
density (whose potential on the sphere is lambda_0).  The paper discretises by Galerkin on meshes and adds the
near-singular part as a sparse correction; on a sphere a diagonal correction of this kind is the reading used
here (listed with the other readings in the design notes).

``single_layer_eigenvalue`` evaluates the defining integral itself: for the zonal harmonic P_n(cos alpha)
about a point x of the sphere of radius a, polar coordinates centred at x give |x - y| = 2a sin(alpha/2) and
dS = a^2 sin(alpha) d(alpha) d(beta), so the singularity cancels and

    lambda_n = (a/2) int_0^pi exp(2ika sin(alpha/2)) cos(alpha/2) P_n(cos alpha) d(alpha),

a smooth integral taken here by Gauss-Legendre quadrature with enough nodes for spectral accuracy.
"""
from __future__ import annotations

import math

import numpy as np

from . import LAPLACE, dense_rows, gauss_legendre, legendre_p


def single_layer_eigenvalue(n: int, k: float = 0.0, radius: float = 1.0) -> complex:
    """lambda_n from the polar-coordinate integral above (k = 0: Laplace)."""
    a = float(radius)
    m = int(2.0 * abs(k) * a + n + 64)
    t, wt = gauss_legendre(m)                      # nodes on [-1, 1] -> alpha in [0, pi]
    al = 0.5 * math.pi * (t + 1.0)
    acc = 0.0 + 0.0j
    for q in range(m):
        P = legendre_p(n, math.cos(al[q]))[n]
        acc += wt[q] * np.exp(2j * k * a * math.sin(0.5 * al[q])) * math.cos(0.5 * al[q]) * P
    return complex(0.5 * a * 0.5 * math.pi * acc)


def green_matrix(X, kernel: int, k: float) -> np.ndarray:
    """G(x_i, x_j) for all node pairs, zero on coincident pairs (FP64 complex, n x n)."""
    D = X[:, None, :] - X[None, :, :]
    r = np.sqrt(np.einsum("ijk,ijk->ij", D, D))
    zero = r == 0.0
    r[zero] = 1.0
    G = (1.0 / (4.0 * math.pi * r)).astype(np.complex128)
    if kernel != LAPLACE:
        G *= np.exp(1j * k * r)
    G[zero] = 0.0
    return G


def single_layer_matrix(X, w, kernel: int, k: float, radius: float = 1.0) -> np.ndarray:
    """The Nystrom matrix A above (dense FP64 complex, n x n)."""
    A = green_matrix(X, kernel, k) * np.asarray(w, dtype=np.float64)[None, :]
    lam0 = single_layer_eigenvalue(0, k if kernel != LAPLACE else 0.0, radius)
    A[np.diag_indices_from(A)] = lam0 - A.sum(axis=1)
    return A


def single_layer_rows(X, w, sigma, kernel: int, k: float, radius: float, rows) -> np.ndarray:
    """(A sigma)_i on sampled rows without forming A: punctured Green sums of w o sigma and of w (the oracle's
    dense sums), then the diagonal term."""
    w = np.asarray(w, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.complex128)
    s = dense_rows(X, X, w * sigma, kernel, k, rows)
    g = dense_rows(X, X, w.astype(np.complex128), kernel, k, rows)
    lam0 = single_layer_eigenvalue(0, k if kernel != LAPLACE else 0.0, radius)
    return s + (lam0 - g) * sigma[np.asarray(rows)]


def solve_dense(X, w, f, kernel: int, k: float, radius: float = 1.0) -> np.ndarray:
    """sigma = A^{-1} f by LU (numpy), FP64."""
    return np.linalg.solve(single_layer_matrix(X, w, kernel, k, radius), np.asarray(f, dtype=np.complex128))


def exact_density(harmonics, kernel: int, k: float, radius: float = 1.0) -> np.ndarray:
    """The exact density of data given as a sum of spherical harmonics: each term divided by lambda_n."""
    kk = k if kernel != LAPLACE else 0.0
    return sum(v / single_layer_eigenvalue(deg, kk, radius) for deg, v in harmonics)


def legendre_table(n_max: int, t) -> np.ndarray:
    """P_0..P_{n_max} at every t (Bonnet's recurrence), shape (n_max + 1, len(t))."""
    t = np.asarray(t, dtype=np.float64)
    P = np.zeros((n_max + 1, t.size))
    P[0] = 1.0
    if n_max >= 1:
        P[1] = t
    for n in range(1, n_max):
        P[n + 1] = ((2 * n + 1) * t * P[n] - n * P[n - 1]) / (n + 1)
    return P


def legendre_projection(g, n_max: int, m: int) -> np.ndarray:
    """Coefficients f_n = (2n+1)/2 int_{-1}^{1} g(t) P_n(t) dt of a function of t = cos(angle), n <= n_max,
    by m-node Gauss-Legendre quadrature (exact for polynomial g of degree < 2m - n_max)."""
    t, wt = gauss_legendre(m)
    P = legendre_table(n_max, t)
    gt = np.asarray(g(t), dtype=np.complex128)
    return np.array([(2 * n + 1) / 2.0 * np.dot(wt * gt, P[n]) for n in range(n_max + 1)])


def zonal_exact_density(X, axis, g, kernel: int, k: float, radius: float, n_max: int, m: int) -> np.ndarray:
    """The exact density for boundary data that depend only on the angle to ``axis`` (data g(cos angle) on
    the sphere of the given radius about the origin): sigma = sum_n f_n / lambda_n P_n, with the data's
    Legendre coefficients f_n by projection and lambda_n by the defining integral."""
    kk = k if kernel != LAPLACE else 0.0
    f = legendre_projection(g, n_max, m)
    ax = np.asarray(axis, dtype=np.float64)
    t = np.clip(X @ (ax / np.linalg.norm(ax)) / np.linalg.norm(X, axis=1), -1.0, 1.0)
    P = legendre_table(n_max, t)
    lam = np.array([single_layer_eigenvalue(n, kk, radius) for n in range(n_max + 1)])
    return (f / lam) @ P


def source_data(x0, radius: float = 1.0):
    """g(t) for the data 1/(4 pi |x - x0|) on the sphere, t the cosine of the angle between x and x0."""
    a, r0 = float(radius), float(np.linalg.norm(x0))
    return lambda t: 1.0 / (4.0 * math.pi * np.sqrt(a * a + r0 * r0 - 2.0 * a * r0 * t))


def plane_wave_data(k: float, radius: float = 1.0):
    """g(t) for the data -exp(i k d.x) on the sphere, t the cosine of the angle between x and d."""
    return lambda t: -np.exp(1j * k * float(radius) * t)
