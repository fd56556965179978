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
