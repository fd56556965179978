"""Pins of the boundary-integral oracle (single-layer equation on a sphere, paper Sec. 4.2) and CPU checks of
the harness's host logic (its closed-form eigenvalues and its GMRES).

The oracle's eigenvalues come from the defining surface integral in polar coordinates; they are pinned here
to closed forms (Laplace a/(2n+1), Helmholtz i k a^2 j_n(ka) h_n(ka) with the oracle's own spherical Hankel
recurrence, sin(ka) e^{ika}/k for n = 0) and to the Laplace limit.  The Nystrom matrix is pinned by its
action on spherical harmonics (second-order convergence to lambda_n Y_n), by the closed-form density of
harmonic data, and by the two independent routes to its rows (numpy Green matrix, the C dense sums).
"""
import math

import numpy as np
import pytest

import ffm_workloads as W


@pytest.fixture(scope="module")
def bie(orc):
    import oracle.bie as B
    return B


@pytest.mark.parametrize("a", [1.0, 0.37])
def test_eigenvalue_laplace_closed_form(bie, a):
    for n in range(0, 8):
        assert abs(bie.single_layer_eigenvalue(n, 0.0, a) - a / (2 * n + 1)) < 1e-13


@pytest.mark.parametrize("k,a", [(0.5, 1.0), (5.0, 1.0), (20.0, 1.0), (13.0, 0.6), (60.0, 1.0)])
def test_eigenvalue_helmholtz_closed_form(orc, bie, k, a):
    z = k * a
    lam0 = math.sin(z) * complex(math.cos(z), math.sin(z)) / k
    assert abs(bie.single_layer_eigenvalue(0, k, a) - lam0) < 1e-13 * max(1.0, abs(lam0) * 1e3)
    # i k a^2 j_n h_n with the oracle's upward Hankel recurrence (stable for n < z; j_n = Re h_n)
    h = orc.sph_hankel1(8, z)
    for n in range(0, 9):
        if n >= z:
            break
        ref = 1j * k * a * a * h[n].real * h[n]
        got = bie.single_layer_eigenvalue(n, k, a)
        assert abs(got - ref) <= 1e-11 * abs(h[n]) * k * a * a, (n, got, ref)


def test_eigenvalue_small_k_limit(bie):
    """lambda_n(k) = 1/(2n+1) + O(k) as k -> 0 (the O(k) term is i k delta_{n0} to first order)."""
    for k in (1e-3, 1e-5):
        for n in range(0, 5):
            lam = bie.single_layer_eigenvalue(n, k)
            assert abs(lam - 1.0 / (2 * n + 1) - (1j * k if n == 0 else 0.0)) < 2 * k * k


def test_harness_eigenvalue_matches_oracle(bie):
    """The harness's closed form (host code of the product package) against the oracle's integral."""
    from paper_1909_05600_amd.bie import single_layer_eigenvalue as lam
    for k, a in ((0.0, 1.0), (0.0, 2.5), (3.0, 1.0), (20.0, 1.0), (177.0, 1.0), (9.0, 0.4)):
        for n in (0, 1, 2, 3, 7, 12):
            ref = bie.single_layer_eigenvalue(n, k, a)
            assert abs(lam(n, k, a) - ref) <= 1e-10 * max(abs(ref), 1e-3 / max(k, 1.0)), (k, a, n)


def test_reduced_grid_moments():
    """The reduced sphere grid integrates low-degree polynomials exactly: area 4 pi a^2, second moments
    4 pi a^4 / 3, and int (xyz)^2 dS = 4 pi a^8 / 105."""
    for nt, a in ((12, 1.0), (40, 1.0), (33, 0.7)):
        X, w = W.reduced_sphere_grid(nt, a)
        assert np.allclose(np.linalg.norm(X, axis=1), a, rtol=0, atol=1e-15)
        assert abs(w.sum() - 4 * math.pi * a * a) < 1e-12
        for c in range(3):
            assert abs(np.dot(w, X[:, c] ** 2) - 4 * math.pi * a ** 4 / 3) < 1e-12
            assert abs(np.dot(w, X[:, c])) < 1e-12
        x, y, z = X.T
        assert abs(np.dot(w, (x * y * z) ** 2) - 4 * math.pi * a ** 8 / 105) < 1e-12


def _harmonic_residual(bie, nt, kernel, k):
    p = W.bie_sphere(nt, kernel, k)
    A = bie.single_layer_matrix(p.X, p.w, kernel, k, p.radius)
    out = []
    for deg, v in p.harmonics:
        lam = bie.single_layer_eigenvalue(deg, k if kernel else 0.0)
        out.append(np.linalg.norm(A @ v - lam * v) / np.linalg.norm(lam * v))
    return np.array(out)


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 4.0), (1, 12.0)])
def test_nystrom_matrix_second_order(bie, kernel, k):
    """A Y_n -> lambda_n Y_n at second order in the node spacing (node counts 4x apart: error ratio > 3)."""
    e1 = _harmonic_residual(bie, 20, kernel, k)
    e2 = _harmonic_residual(bie, 40, kernel, k)
    print("harmonic residuals", e1, e2)
    assert np.all(e2[1:] < e1[1:] / 3.0)
    assert np.all(e2 < 2e-3)
    assert e1[0] < 1e-13 and e2[0] < 1e-13          # the constant density is exact by construction


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 5.0)])
def test_dense_solve_converges_to_closed_form(bie, kernel, k):
    errs = []
    for nt in (16, 32):
        p = W.bie_sphere(nt, kernel, k)
        s = bie.solve_dense(p.X, p.w, p.f, kernel, k, p.radius)
        ex = bie.exact_density(p.harmonics, kernel, k, p.radius)
        sw = np.sqrt(p.w)
        errs.append(np.linalg.norm((s - ex) * sw) / np.linalg.norm(ex * sw))
    print("dense solve vs closed form", errs)
    assert errs[1] < errs[0] / 3.0 and errs[1] < 5e-4


def test_rows_match_matrix(bie):
    """single_layer_rows (the C dense sums) equals rows of single_layer_matrix (numpy Green matrix)."""
    p = W.bie_sphere(14, 1, 7.0)
    rng = np.random.default_rng(3)
    sig = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    rows = np.arange(0, p.n, 7)
    A = bie.single_layer_matrix(p.X, p.w, 1, 7.0)
    got = bie.single_layer_rows(p.X, p.w, sig, 1, 7.0, 1.0, rows)
    assert np.allclose(got, (A @ sig)[rows], rtol=1e-12, atol=1e-14)


def test_gmres_host_logic_dense(bie):
    """The harness's GMRES on CPU tensors with a dense FP64 operator: the oracle's Nystrom matrix and a random
    non-normal matrix; restarts, monotone residual estimates, the true residual, zero data and the cap."""
    import torch
    from paper_1909_05600_amd.bie import gmres
    p = W.bie_sphere(12, 1, 6.0)
    A = torch.from_numpy(bie.single_layer_matrix(p.X, p.w, 1, 6.0))
    b = torch.from_numpy(p.f.astype(np.complex128))
    for restart in (200, 7):
        x, info = gmres(lambda v: A @ v, b, tol=1e-10, restart=restart, maxiter=2000)
        assert info["converged"], info["iterations"]
        r = info["residuals"]
        if restart == 200:
            assert all(r[i + 1] <= r[i] * (1 + 1e-9) for i in range(len(r) - 1))
        assert float(torch.linalg.vector_norm(A @ x - b) / torch.linalg.vector_norm(b)) < 1e-9
        ref = np.linalg.solve(A.numpy(), b.numpy())
        assert np.linalg.norm(x.numpy() - ref) / np.linalg.norm(ref) < 1e-7
    rng = np.random.default_rng(1)
    M = torch.from_numpy(np.eye(60) * 3 + rng.standard_normal((60, 60)) / 8 + 1j * np.triu(
        rng.standard_normal((60, 60))) / 5)
    c = torch.from_numpy(rng.standard_normal(60) + 0j)
    x, info = gmres(lambda v: M @ v, c, tol=1e-12, restart=10, maxiter=500)
    assert info["converged"]
    assert np.allclose(x.numpy(), np.linalg.solve(M.numpy(), c.numpy()), rtol=0, atol=1e-10)
    x, info = gmres(lambda v: M @ v, torch.zeros(60, dtype=torch.complex128))
    assert info["converged"] and info["iterations"] == 0 and not torch.any(x)
    x, info = gmres(lambda v: M @ v, c, tol=1e-14, restart=3, maxiter=5)
    assert info["iterations"] == 5 and not info["converged"]


def test_legendre_projection_closed_forms(orc, bie):
    """Projection coefficients of the zonal data: a point charge at r0 < a gives r0^n / (4 pi a^(n+1)); the
    plane wave -exp(i k a t) gives -(2n+1) i^n j_n(ka) (j_n as the real part of the oracle's Hankel
    recurrence below the turning point, scipy's spherical_jn above it)."""
    import scipy.special as sp
    a, r0 = 1.3, 0.6
    f = bie.legendre_projection(bie.source_data(np.array([0.0, r0, 0.0]), a), 40, 120)
    ref = np.array([r0 ** n / (4 * math.pi * a ** (n + 1)) for n in range(41)])
    # FP64 rounding of the quadrature sums: (2n+1)/2 x |g| ~ 4e1 x 0.1 x 2^-53 x sqrt(m) ~ 1e-14 at most
    assert np.allclose(f, ref, rtol=1e-12, atol=1e-14)
    k = 17.0
    f = bie.legendre_projection(bie.plane_wave_data(k, a), 60, 160)
    z = k * a
    h = orc.sph_hankel1(60, z)
    for n in range(61):
        jn = h[n].real if n < z else sp.spherical_jn(n, z)
        assert abs(f[n] + (2 * n + 1) * (1j ** n) * jn) < 1e-12 * (2 * n + 1), n


@pytest.mark.parametrize("data", ["source", "plane_wave"])
def test_zonal_series_reconstructs_data(bie, data):
    """sum_n f_n P_n(cos angle) equals the boundary data at the nodes (the projection and the Legendre
    table at the nodes together)."""
    p = W.bie_sphere(24, 1, 9.0, data=data)
    if data == "source":
        g, ax, nmax = bie.source_data(p.x0, p.radius), p.x0, 60
    else:
        g, ax, nmax = bie.plane_wave_data(p.k, p.radius), p.direction, 50
    f = bie.legendre_projection(g, nmax, 160)
    t = p.X @ (ax / np.linalg.norm(ax)) / np.linalg.norm(p.X, axis=1)
    assert np.allclose(f @ bie.legendre_table(nmax, t), p.f, rtol=0, atol=1e-12)


def test_harness_closed_forms_match_oracle(bie):
    """The harness's closed-form densities (point source coefficients, the stable plane-wave series) against
    the oracle's projection-and-integral densities."""
    from paper_1909_05600_amd import bie as hb
    p = W.bie_sphere(20, 0, data="source")
    ref = bie.zonal_exact_density(p.X, p.x0, bie.source_data(p.x0, p.radius), 0, 0.0, p.radius, 60, 120)
    got = hb.zonal_density(p.X, p.x0, hb.point_source_coefficients(np.linalg.norm(p.x0), p.radius))
    print("source density: harness vs oracle %.2e" % (np.linalg.norm(got - ref) / np.linalg.norm(ref)))
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-10
    for k in (3.0, 20.0):
        p = W.bie_sphere(20, 1, k, data="plane_wave")
        ref = bie.zonal_exact_density(p.X, p.direction, bie.plane_wave_data(k, p.radius), 1, k, p.radius,
                                      int(k) + 40, 2 * int(k) + 120)
        got = hb.plane_wave_density(p.X, p.direction, k, p.radius)
        print("plane wave k=%g: harness vs oracle %.2e" % (k, np.linalg.norm(got - ref) / np.linalg.norm(ref)))
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-10, k


@pytest.mark.parametrize("kernel,k,data", [(0, 0.0, "source"), (1, 5.0, "plane_wave"), (1, 5.0, "source")])
def test_dense_solve_converges_zonal(bie, kernel, k, data):
    errs = []
    for nt in (16, 32):
        p = W.bie_sphere(nt, kernel, k, data=data)
        s = bie.solve_dense(p.X, p.w, p.f, kernel, k, p.radius)
        if data == "source":
            ex = bie.zonal_exact_density(p.X, p.x0, bie.source_data(p.x0, p.radius), kernel, k, p.radius, 60, 120)
        else:
            ex = bie.zonal_exact_density(p.X, p.direction, bie.plane_wave_data(k, p.radius), kernel, k,
                                         p.radius, 50, 140)
        sw = np.sqrt(p.w)
        errs.append(np.linalg.norm((s - ex) * sw) / np.linalg.norm(ex * sw))
    print("dense solve vs closed form (%s)" % data, errs)
    assert errs[1] < errs[0] / 3.0 and errs[1] < 2e-3
