"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.py.

This module only draws random numbers and assembles arrays: it holds none of
the method's arithmetic.  Every generator uses numpy's PCG64 stream
(``numpy.random.default_rng(seed)``) so the same seed gives the same arrays on
every machine with the same numpy.

Workloads follow the paper's scalability experiments (Section 4.1): random
nodes on the unit sphere, the same set used as sources and targets, a
prescribed accuracy of 1e-3 on the matrix-vector product.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

LAPLACE = 0
HELMHOLTZ = 1


def sphere_points(n: int, rng: np.random.Generator) -> np.ndarray:
    """n points uniform on the unit sphere: normalised standard Gaussians (FP64, n x 3)."""
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def cube_points(n: int, rng: np.random.Generator, centre, edge: float) -> np.ndarray:
    """n points uniform in an axis-aligned cube of the given centre and edge."""
    return np.asarray(centre, dtype=np.float64) + (rng.random((n, 3)) - 0.5) * edge


def ellipsoid_points(n: int, rng: np.random.Generator, axes=(0.25, 0.5, 1.0)) -> np.ndarray:
    """Sphere points scaled by the semi-axes (axis ratio 1:2:4); the density is non-uniform."""
    return sphere_points(n, rng) * np.asarray(axes, dtype=np.float64)


def wavenumber_10ppw(n: int) -> float:
    """k giving about ten points per wavelength for n points on the unit sphere."""
    return 2.0 * math.pi * math.sqrt(n / (4.0 * math.pi)) / 10.0


@dataclass
class Workload:
    name: str
    X: np.ndarray                 # targets, FP64 (n_x, 3)
    Y: np.ndarray                 # sources, FP64 (n_y, 3); the same object as X when the sets coincide
    kernel: int                   # LAPLACE or HELMHOLTZ
    k: float
    eps: float
    wu: np.ndarray                # w*u in source order: float64 (real) or complex64/complex128
    rows: np.ndarray | None = None   # sampled target indices for error checks
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.X.shape[0])


def laplace_sphere(n: int = 4096, seed: int = 1, eps: float = 1e-3) -> Workload:
    """Laplace, same set for sources and targets on the unit sphere, w = 4*pi/N, u ~ N(0,1) FP64."""
    rng = np.random.default_rng(seed)
    X = sphere_points(n, rng)
    u = rng.standard_normal(n)
    wu = (4.0 * math.pi / n) * u
    return Workload("laplace_sphere_%d" % n, X, X, LAPLACE, 0.0, eps, wu,
                    rows=np.arange(n) if n <= 4096 else np.sort(rng.choice(n, 4096, replace=False)))


def helmholtz_sphere(n: int = 1 << 20, seed: int = 2, eps: float = 1e-3, k: float | None = None,
                     n_rows: int = 4096) -> Workload:
    """Helmholtz, unit sphere, k for ~10 points per wavelength, complex64 u (Re, Im ~ N(0,1)), w = 4*pi/N."""
    rng = np.random.default_rng(seed)
    X = sphere_points(n, rng)
    u = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    wu = (u * np.float32(4.0 * math.pi / n)).astype(np.complex64)
    kk = wavenumber_10ppw(n) if k is None else float(k)
    rows = np.sort(rng.choice(n, min(n_rows, n), replace=False))
    return Workload("helmholtz_sphere_%d" % n, X, X, HELMHOLTZ, kk, eps, wu, rows=rows)


def sphere_plus_cube(n: int = 10_000_000, seed: int = 3, eps: float = 1e-3, n_rows: int = 4096,
                     cube_frac: float = 0.2) -> Workload:
    """Helmholtz on a sphere plus a cube cluster (edge 0.5, centre ~ U[-0.75, 0.75]^3): a non-uniform octree."""
    rng = np.random.default_rng(seed)
    n_cube = int(round(n * cube_frac))
    n_sph = n - n_cube
    P = sphere_points(n_sph, rng)
    centre = rng.uniform(-0.75, 0.75, size=3)
    C = cube_points(n_cube, rng, centre, 0.5)
    X = np.concatenate([P, C], axis=0)
    u = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    wu = (u * np.float32(4.0 * math.pi / n)).astype(np.complex64)
    kk = wavenumber_10ppw(n_sph)
    rows = np.sort(rng.choice(n, min(n_rows, n), replace=False))
    return Workload("sphere_cube_%d" % n, X, X, HELMHOLTZ, kk, eps, wu, rows=rows,
                    meta={"n_sphere": n_sph, "cube_centre": centre.tolist()})


def batched_instances(count: int = 256, seed: int = 4, n_min: int = 2000, n_max: int = 200_000,
                      eps: float = 1e-3) -> list[Workload]:
    """Independent instances: N log-uniform in [n_min, n_max]; even = Laplace, odd = Helmholtz with
    k log-uniform in [1, 50]; geometry cycles sphere / ellipsoid (1:2:4) / cube [-1, 1]^3."""
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        geo = i % 3
        if geo == 0:
            X = sphere_points(n, rng)
        elif geo == 1:
            X = ellipsoid_points(n, rng)
        else:
            X = cube_points(n, rng, (0.0, 0.0, 0.0), 2.0)
        kern = LAPLACE if i % 2 == 0 else HELMHOLTZ
        k = 0.0 if kern == LAPLACE else float(math.exp(rng.uniform(0.0, math.log(50.0))))
        u = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
        wu = (u * np.float32(4.0 * math.pi / n)).astype(np.complex64)
        rows = np.sort(rng.choice(n, min(256, n), replace=False))
        out.append(Workload("inst%03d" % i, X, X, kern, k, eps, wu, rows=rows,
                            meta={"geometry": ("sphere", "ellipsoid", "cube")[geo]}))
    return out


def serving_plans(count: int = 64, seed: int = 5, n_min: int = 10_000, n_max: int = 5_000_000,
                  eps: float = 1e-3, scale: float = 1.0) -> list[Workload]:
    """Resident plans for the serving workload: N log-uniform in [n_min, n_max] (times ``scale``),
    kernel alternating, Helmholtz k by the ten-points-per-wavelength rule, geometry cycling."""
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        n = max(64, int(round(scale * math.exp(rng.uniform(math.log(n_min), math.log(n_max))))))
        geo = i % 3
        if geo == 0:
            X = sphere_points(n, rng)
        elif geo == 1:
            X = ellipsoid_points(n, rng)
        else:
            X = cube_points(n, rng, (0.0, 0.0, 0.0), 2.0)
        kern = LAPLACE if i % 2 == 0 else HELMHOLTZ
        k = 0.0 if kern == LAPLACE else wavenumber_10ppw(n)
        u = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
        wu = (u * np.float32(4.0 * math.pi / n)).astype(np.complex64)
        out.append(Workload("plan%02d" % i, X, X, kern, k, eps, wu,
                            meta={"geometry": ("sphere", "ellipsoid", "cube")[geo]}))
    return out


def poisson_arrivals(n_sessions: int, rate: float, seed: int = 5) -> np.ndarray:
    """Session start times (seconds) of a Poisson process of the given rate."""
    rng = np.random.default_rng([seed, 99991])
    return np.cumsum(rng.exponential(1.0 / rate, size=n_sessions))


def shell_grid(n_theta: int, n_phi: int, radius: float = 1.0):
    """Product Gauss-Legendre (in cos theta) x trapezoid (in phi) nodes on a sphere of the given radius,
    with the area weights of that product rule.  Used as the source set of the uniform-shell closed forms."""
    ct, wt = np.polynomial.legendre.leggauss(n_theta)
    ph = 2.0 * math.pi * np.arange(n_phi) / n_phi
    st = np.sqrt(1.0 - ct * ct)
    P = np.stack([np.outer(st, np.cos(ph)).ravel(), np.outer(st, np.sin(ph)).ravel(),
                  np.repeat(ct, n_phi)], axis=1) * radius
    w = np.repeat(wt, n_phi) * (2.0 * math.pi / n_phi) * radius * radius
    return P, w


def reduced_sphere_grid(n_theta: int, radius: float = 1.0):
    """Quasi-uniform quadrature nodes on a sphere: n_theta Gauss-Legendre rings in cos(theta); ring m holds
    max(6, ceil(2 n_theta sin(theta_m))) equispaced azimuths, every other ring turned by half a step.  A node's
    weight is its ring's Gauss weight times 2 pi over the ring's azimuth count, times radius^2.  About
    4 n_theta^2 / pi nodes, spaced evenly over the surface like the vertices of a uniform surface mesh."""
    ct, wt = np.polynomial.legendre.leggauss(n_theta)
    st = np.sqrt(1.0 - ct * ct)
    n_phi = np.maximum(6, np.ceil(2.0 * n_theta * st).astype(np.int64))
    ring = np.repeat(np.arange(n_theta), n_phi)
    start = np.concatenate([[0], np.cumsum(n_phi)[:-1]])
    j = np.arange(int(n_phi.sum())) - np.repeat(start, n_phi)
    ph = 2.0 * math.pi * (j + 0.5 * (ring % 2)) / n_phi[ring]
    P = np.stack([st[ring] * np.cos(ph), st[ring] * np.sin(ph), ct[ring]], axis=1) * radius
    w = wt[ring] * (2.0 * math.pi / n_phi[ring]) * radius * radius
    return P, w


def n_theta_for(n: int) -> int:
    """The ring count whose reduced sphere grid holds about n nodes."""
    return max(4, int(round(math.sqrt(math.pi * n / 4.0))))


@dataclass
class SurfaceProblem:
    """A Dirichlet problem on a sphere for the single-layer equation: nodes, weights and boundary data f.
    ``data`` names the data: "harmonics" (a sum of spherical harmonics, each term's degree and nodal values
    in ``harmonics``), "source" (the potential 1/(4 pi |x - x0|) of a unit point charge at ``x0`` inside the
    sphere) or "plane_wave" (f = -exp(i k d.x), a sound-soft sphere hit by a plane wave along ``direction``)."""
    name: str
    X: np.ndarray                 # nodes, FP64 (n, 3)
    w: np.ndarray                 # quadrature weights, FP64 (n,)
    kernel: int
    k: float
    eps: float
    radius: float
    data: str
    f: np.ndarray                 # boundary data at the nodes (complex128)
    harmonics: list = field(default_factory=list)   # [(degree, values at the nodes, FP64)]
    x0: np.ndarray | None = None
    direction: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.X.shape[0])


def bie_sphere(n_theta: int, kernel: int = HELMHOLTZ, k: float | None = None, eps: float = 1e-3,
               radius: float = 1.0, data: str = "harmonics") -> SurfaceProblem:
    """A single-layer problem on the reduced sphere grid of radius a.  Helmholtz k defaults to ten nodes per
    wavelength.  Data: "harmonics" is f = 1 + x/a + xyz/a^3 (degrees 0, 1, 3: x and xyz are harmonic
    polynomials); "source" puts the charge at x0 = (0.15, -0.25, 0.35) a; "plane_wave" travels along
    d = (1, 2, 3)/sqrt(14)."""
    X, w = reduced_sphere_grid(n_theta, radius)
    x, y, z = (X / radius).T
    kk = 0.0 if kernel == LAPLACE else (wavenumber_10ppw(X.shape[0]) / radius if k is None else float(k))
    name = "bie_sphere_%s_%d" % (data, X.shape[0])
    if data == "harmonics":
        h = [(0, np.ones_like(x)), (1, x.copy()), (3, x * y * z)]
        return SurfaceProblem(name, X, w, kernel, kk, eps, radius, data, sum(v for _, v in h).astype(complex),
                              harmonics=h)
    if data == "source":
        x0 = np.array([0.15, -0.25, 0.35]) * radius
        f = (1.0 / (4.0 * math.pi * np.linalg.norm(X - x0, axis=1))).astype(np.complex128)
        return SurfaceProblem(name, X, w, kernel, kk, eps, radius, data, f, x0=x0)
    if data == "plane_wave":
        if kernel != HELMHOLTZ:
            raise ValueError("plane-wave data needs the Helmholtz kernel")
        d = np.array([1.0, 2.0, 3.0]) / math.sqrt(14.0)
        f = -np.exp(1j * kk * (X @ d))
        return SurfaceProblem(name, X, w, kernel, kk, eps, radius, data, f, direction=d)
    raise ValueError("unknown data %r" % data)
