"""Boundary-integral use of the FFM product: the single-layer equation on a sphere, solved by GMRES with one
FFM product per iteration.

Sec. 4.2 of the paper solves S sigma = f for Dirichlet data with a Galerkin discretisation on surface meshes:
the dense part of the matrix is the free-space Green kernel between quadrature nodes, applied by the FFM, and
the near-singular part is a sparse correction added to it.  This module keeps that split on a sphere with the
unknowns on the quadrature nodes themselves (a Nystrom discretisation):

    (A sigma)_i = sum_{j != i} G(x_i, x_j) w_j sigma_j  +  c_i sigma_i,

where the sum is the FFM product of w o sigma (coincident nodes contribute nothing to it) and the diagonal
correction is singularity subtraction against the constant density, whose single-layer potential on the
sphere is the closed form lambda_0:

    c_i = lambda_0 - sum_{j != i} G(x_i, x_j) w_j     (one FFM product, at set-up).

Hence (A sigma)_i = sum_{j != i} G_ij w_j (sigma_j - sigma_i) + lambda_0 sigma_i: the integrand vanishes at
the singular point and the rule is second-order accurate on a quasi-uniform grid.

Spherical harmonics of degree n are eigenfunctions of the single-layer operator on a sphere of radius a, with
eigenvalue a / (2n + 1) for the Laplace kernel 1/(4 pi r) and i k a^2 j_n(ka) h_n(ka) for the Helmholtz
kernel e^{ikr}/(4 pi r); ``single_layer_eigenvalue`` returns them, so the exact density of harmonic data is
known in closed form.

The FFM product runs in the HIP library through its C ABI; the solver's vector operations (Gram-Schmidt on
the Krylov basis, the diagonal term) are plain device tensor operations, and the small Hessenberg least-squares
problem is solved on the host in FP64.
"""
from __future__ import annotations

import math

import numpy as np

from . import FFM_HELMHOLTZ, FFM_LAPLACE, Plan


def single_layer_eigenvalue(n: int, k: float = 0.0, radius: float = 1.0) -> complex:
    """Eigenvalue of the single-layer operator for degree-n spherical harmonics on a sphere of the given
    radius; k = 0 is the Laplace kernel 1/(4 pi r), k > 0 the Helmholtz kernel e^{ikr}/(4 pi r)."""
    if n < 0:
        raise ValueError("degree must be >= 0")
    a = float(radius)
    if k == 0.0:
        return complex(a / (2 * n + 1))
    from scipy.special import spherical_jn, spherical_yn
    z = k * a
    j = float(spherical_jn(n, z))
    y = float(spherical_yn(n, z))
    return complex(1j * k * a * a * j * (j + 1j * y))


def _legendre_sum(t, coeffs):
    """sum_n coeffs[n] P_n(t) for an array t, by Bonnet's recurrence."""
    t = np.asarray(t, dtype=np.float64)
    p0, p1 = np.ones_like(t), t.copy()
    acc = coeffs[0] * p0
    if len(coeffs) > 1:
        acc = acc + coeffs[1] * p1
    for n in range(1, len(coeffs) - 1):
        p0, p1 = p1, ((2 * n + 1) * t * p1 - n * p0) / (n + 1)
        acc = acc + coeffs[n + 1] * p1
    return acc


def zonal_density(X, axis, coeffs, k: float = 0.0, radius: float = 1.0, centre=(0.0, 0.0, 0.0)):
    """Exact density for zonal data f = sum_n coeffs[n] P_n(cos g), g the angle between x - centre and
    ``axis``: sigma = sum_n coeffs[n] / lambda_n P_n(cos g) (host, FP64; X a host array)."""
    Xc = np.asarray(X, dtype=np.float64) - np.asarray(centre, dtype=np.float64)
    ax = np.asarray(axis, dtype=np.float64)
    t = np.clip(Xc @ (ax / np.linalg.norm(ax)) / np.linalg.norm(Xc, axis=1), -1.0, 1.0)
    c = [coeffs[n] / single_layer_eigenvalue(n, k, radius) for n in range(len(coeffs))]
    return _legendre_sum(t, np.asarray(c, dtype=np.complex128))


def point_source_coefficients(r0: float, radius: float = 1.0, tol: float = 1e-17):
    """Legendre coefficients of 1/(4 pi |x - x0|) on a sphere of radius a about a charge at distance r0 < a
    from the centre: r0^n / (4 pi a^(n+1)), up to the first degree below tol."""
    a = float(radius)
    q = float(r0) / a
    if not 0.0 <= q < 1.0:
        raise ValueError("the charge must lie inside the sphere")
    n_max = 0 if q == 0.0 else int(math.log(tol) / math.log(q)) + 1
    return np.array([q ** n / (4.0 * math.pi * a) for n in range(n_max + 1)], dtype=np.complex128)


def plane_wave_density(X, direction, k: float, radius: float = 1.0, centre=(0.0, 0.0, 0.0)):
    """Exact density for the sound-soft sphere under a plane wave, data f = -exp(i k d.x): the Legendre
    coefficients of the data are -(2n+1) i^n j_n(ka) exp(i k d.centre), and dividing by lambda_n = i k a^2
    j_n h_n leaves -(2n+1) i^n / (i k a^2 h_n(ka)), evaluated in that stable form."""
    from scipy.special import spherical_jn, spherical_yn
    a, z = float(radius), float(k) * float(radius)
    n_max = int(z + 10.0 * z ** (1.0 / 3.0) + 20)
    n = np.arange(n_max + 1)
    h = spherical_jn(n, z) + 1j * spherical_yn(n, z)
    phase = np.exp(1j * k * (np.asarray(centre, dtype=np.float64) @ np.asarray(direction, dtype=np.float64)
                             / np.linalg.norm(direction)))
    c = -(2 * n + 1) * (1j ** n) / (1j * k * a * a * h) * phase
    Xc = np.asarray(X, dtype=np.float64) - np.asarray(centre, dtype=np.float64)
    d = np.asarray(direction, dtype=np.float64)
    t = np.clip(Xc @ (d / np.linalg.norm(d)) / np.linalg.norm(Xc, axis=1), -1.0, 1.0)
    return _legendre_sum(t, c)


class SingleLayer:
    """The discrete single-layer operator A of a sphere (radius ``radius``, any centre) on the nodes X with
    quadrature weights w: ``matvec(sigma)`` is one FFM product plus the diagonal correction.

    X: CUDA float64 (n, 3) nodes on the sphere; w: (n,) weights (any float dtype, host or device).
    Extra keyword arguments go to the FFM plan (precision, transforms, ...).
    """

    def __init__(self, X, w, kernel: int, k: float, eps: float, radius: float = 1.0, **plan_kw):
        import torch
        if kernel not in (FFM_LAPLACE, FFM_HELMHOLTZ):
            raise ValueError("kernel must be FFM_LAPLACE or FFM_HELMHOLTZ")
        self.kernel, self.k, self.eps, self.radius = int(kernel), float(k), float(eps), float(radius)
        self.n = int(X.shape[0])
        w = torch.as_tensor(w, device=X.device)
        if w.shape != (self.n,):
            raise ValueError("w must have one weight per node")
        self.w = w.to(torch.float32).contiguous()
        self.plan = Plan(X, X, self.kernel, self.k if self.kernel == FFM_HELMHOLTZ else 0.0, self.eps, **plan_kw)
        self.lambda0 = single_layer_eigenvalue(0, self.k if self.kernel == FFM_HELMHOLTZ else 0.0, self.radius)
        row = self.plan.apply(self.w.to(torch.complex64))          # sum_{j != i} G_ij w_j
        self.diag = (torch.full_like(row, self.lambda0) - row).contiguous()
        self.products = 1

    def matvec(self, sigma, out=None):
        """A sigma for a complex64 device vector sigma (length n)."""
        v = self.plan.apply((sigma * self.w).to(sigma.dtype), out=out)
        v.addcmul_(self.diag, sigma)
        self.products += 1
        return v

    def destroy(self):
        self.plan.destroy()


def gmres(matvec, b, tol: float = 1e-5, restart: int = 50, maxiter: int = 500):
    """Restarted GMRES (Saad and Schultz) for A x = b with x0 = 0.

    The Krylov basis is kept on the device in b's dtype and orthogonalised by classical Gram-Schmidt applied
    twice; the Hessenberg matrix, its Givens rotations and the small triangular solve are FP64 on the host.
    Stops when the residual estimate falls to tol * |b| or after maxiter products.  Returns (x, info) with
    info = {"iterations", "converged", "residuals"} (relative residual estimates, one per iteration)."""
    import torch
    n = b.numel()
    bnorm = float(torch.linalg.vector_norm(b))
    x = torch.zeros_like(b)
    info = {"iterations": 0, "converged": bnorm == 0.0, "residuals": []}
    if n == 0 or bnorm == 0.0:
        return x, info
    m = max(1, min(int(restart), n))
    V = torch.empty((m + 1, n), dtype=b.dtype, device=b.device)
    it = 0
    r = b.clone()
    while it < maxiter:
        if it > 0:
            r = b - matvec(x)
        beta = float(torch.linalg.vector_norm(r))
        if beta <= tol * bnorm:
            info["converged"] = True
            break
        V[0] = r / beta
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.float64)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        j_done = 0
        for j in range(m):
            wv = matvec(V[j])
            Vj = V[:j + 1]
            # V^H w as conj(V conj(w)): no conjugated copy of the basis
            h = torch.mv(Vj, wv.conj()).conj()
            wv = wv - h @ Vj
            h2 = torch.mv(Vj, wv.conj()).conj()
            wv = wv - h2 @ Vj
            hcol = (h + h2).to(torch.complex128).cpu().numpy()
            hn = float(torch.linalg.vector_norm(wv))
            H[:j + 1, j] = hcol
            H[j + 1, j] = hn
            if hn > 0.0:
                V[j + 1] = wv / hn
            for i in range(j):                       # earlier rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a_, b_ = H[j, j], H[j + 1, j]
            den = math.hypot(abs(a_), abs(b_))
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            elif abs(a_) == 0.0:
                cs[j], sn[j] = 0.0, np.conj(b_) / abs(b_)
            else:
                cs[j] = abs(a_) / den
                sn[j] = (a_ / abs(a_)) * np.conj(b_) / den
            H[j, j] = cs[j] * a_ + sn[j] * b_
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            res = abs(g[j + 1]) / bnorm
            info["residuals"].append(float(res))
            if res <= tol or it >= maxiter or hn == 0.0:
                break
        y = np.zeros(j_done, dtype=np.complex128)
        for i in range(j_done - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:j_done]) / H[i, i]
        x = x + torch.from_numpy(y).to(device=b.device, dtype=b.dtype) @ V[:j_done]
        if info["residuals"][-1] <= tol:
            info["converged"] = True
            break
    info["iterations"] = it
    return x, info


def solve(A: SingleLayer, f, tol: float = 1e-5, restart: int = 50, maxiter: int = 500):
    """sigma with A sigma = f (f on the device, any complex or real dtype; solved in complex64)."""
    import torch
    b = torch.as_tensor(f, device=A.w.device).to(torch.complex64).contiguous()
    return gmres(A.matvec, b, tol=tol, restart=restart, maxiter=maxiter)
