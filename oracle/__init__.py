"""FP64 CPU oracle of the Fast Free Memory method (arXiv:1909.05600).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_1909_05600_amd``) and never imports it.

The C library (``ffm_oracle.c``) holds the arithmetic; this module only
marshals numpy arrays.  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ffm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libffm_oracle.so")
_lib = None

LAPLACE = 0
HELMHOLTZ = 1
LAPLACE_DN = 2          # normal derivative at the target: the adjoint double-layer kernel
HELMHOLTZ_DN = 3
LAPLACE_DL = 4          # normal derivative at the source: the double-layer kernel
HELMHOLTZ_DL = 5
LAPLACE_GRAD = 6        # gradient at the target: three components per target
HELMHOLTZ_GRAD = 7


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int32, C.c_double
        sig = {
            "orc_dense_rows": (None, [P, P, i64, P, C.c_int, dbl, P, i64, P]),
            "orc_gauss_legendre": (None, [C.c_int, P, P]),
            "orc_legendre_p": (None, [C.c_int, dbl, P]),
            "orc_sph_hankel1": (None, [C.c_int, dbl, P]),
            "orc_cheb_nodes": (None, [C.c_int, P]),
            "orc_lagrange_basis": (None, [C.c_int, dbl, P]),
            "orc_gegenbauer_rank": (C.c_int, [dbl, dbl, dbl]),
            "orc_sphere_quadrature": (i64, [C.c_int, P, P]),
            "orc_gegenbauer_diag": (None, [C.c_int, dbl, P, P]),
            "orc_plan_create": (P, [P, i64, P, i64, C.c_int, dbl, dbl, P]),
            "orc_plan_free": (None, [P]),
            "orc_apply": (None, [P, P, P, i64]),
            "orc_leaf": (C.c_int, [P]),
            "orc_num_threads": (C.c_int, []),
            "orc_d0": (dbl, [P]),
            "orc_corner": (None, [P, C.c_int, P]),
            "orc_npoints": (i64, [P, C.c_int]),
            "orc_keys": (None, [P, C.c_int, P]),
            "orc_perm": (None, [P, C.c_int, P]),
            "orc_nbox": (i64, [P, C.c_int, C.c_int]),
            "orc_box_start": (None, [P, C.c_int, C.c_int, P]),
            "orc_box_ijk": (None, [P, C.c_int, C.c_int, P]),
            "orc_box_centre": (None, [P, C.c_int, C.c_int, P]),
            "orc_nfar": (i64, [P, C.c_int]),
            "orc_far": (None, [P, C.c_int, P, P, P]),
            "orc_nnear": (i64, [P, C.c_int]),
            "orc_near": (None, [P, C.c_int, P, P]),
            "orc_nearly": (i64, [P, C.c_int]),
            "orc_early": (None, [P, C.c_int, P, P]),
            "orc_level_method": (C.c_int, [P, C.c_int]),
            "orc_level_order": (C.c_int, [P, C.c_int]),
            "orc_grid_forward": (None, [C.c_int, C.c_int, dbl, dbl, dbl, C.c_int, P, P, i64, P]),
            "orc_grid_backward": (None, [C.c_int, C.c_int, dbl, dbl, dbl, C.c_int, P, P, i64, P]),
            "orc_es_hat": (dbl, [C.c_int, dbl, dbl]),
            "orc_aca": (C.c_int, [C.c_int, P, dbl, P, P]),
            "orc_dense_rows_dn": (None, [P, P, i64, P, C.c_int, dbl, P, P, i64, P]),
            "orc_dense_rows_dl": (None, [P, P, i64, P, C.c_int, dbl, P, P, i64, P]),
            "orc_dense_rows_grad": (None, [P, P, i64, P, C.c_int, dbl, P, i64, P]),
            "orc_lagrange_basis_deriv": (None, [C.c_int, dbl, P]),
            "orc_aca_ranks": (C.c_int, [P, C.c_int, dbl, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


MAX_LEVELS = 21


class _Options(C.Structure):
    _fields_ = [("n_leaf", C.c_int32), ("kappa", C.c_double), ("r1_override", C.c_int32),
                ("max_level", C.c_int32), ("grid_p", C.c_int32 * MAX_LEVELS), ("grid_w", C.c_int32 * MAX_LEVELS),
                ("grid_beta", C.c_double * MAX_LEVELS), ("aca_tol", C.c_double), ("aca", C.c_int32 * MAX_LEVELS),
                ("target_normals", C.c_void_p), ("adaptive", C.c_int32), ("source_normals", C.c_void_p)]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _coords(P) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(-1, 3))


def _complex128(wu) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(wu).astype(np.complex128).ravel())


def dense_rows(X, Y, wu, kernel: int, k: float, rows) -> np.ndarray:
    """FP64 direct sum v_i = sum_{j: r_ij > 0} G(x_i - y_j) wu_j on the given target rows (complex128)."""
    X, Y = _coords(X), _coords(Y)
    w = _complex128(wu)
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).ravel())
    out = np.zeros(r.size, dtype=np.complex128)
    lib().orc_dense_rows(_ptr(X), _ptr(Y), Y.shape[0], _ptr(w), int(kernel), float(k), _ptr(r), r.size,
                         _ptr(out))
    return out


def dense_rows_dn(X, Y, wu, kernel: int, k: float, NX, rows) -> np.ndarray:
    """FP64 direct sum of the normal derivative at the targets, v_i = sum_{j: r_ij > 0} n_i . grad_x G(x_i - y_j)
    wu_j (the adjoint double-layer kernel), on the given rows; kernel is the base kernel (0 or 1)."""
    X, Y, N = _coords(X), _coords(Y), _coords(NX)
    w = _complex128(wu)
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).ravel())
    out = np.zeros(r.size, dtype=np.complex128)
    lib().orc_dense_rows_dn(_ptr(X), _ptr(Y), Y.shape[0], _ptr(w), int(kernel) & 1, float(k), _ptr(N), _ptr(r),
                            r.size, _ptr(out))
    return out


def dense_rows_dl(X, Y, wu, kernel: int, k: float, NY, rows) -> np.ndarray:
    """FP64 direct sum of the normal derivative at the sources, v_i = sum_{j: r_ij > 0} n_j . grad_y G(x_i - y_j)
    wu_j (the double-layer kernel), on the given rows; kernel is the base kernel (0 or 1)."""
    X, Y, N = _coords(X), _coords(Y), _coords(NY)
    w = _complex128(wu)
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).ravel())
    out = np.zeros(r.size, dtype=np.complex128)
    lib().orc_dense_rows_dl(_ptr(X), _ptr(Y), Y.shape[0], _ptr(w), int(kernel) & 1, float(k), _ptr(N), _ptr(r),
                            r.size, _ptr(out))
    return out


def dense_rows_grad(X, Y, wu, kernel: int, k: float, rows) -> np.ndarray:
    """FP64 direct sum of the gradient at the targets, v_i = sum_{j: r_ij > 0} grad_x G(x_i - y_j) wu_j, on the
    given rows: complex128 (rows, 3); kernel is the base kernel (0 or 1)."""
    X, Y = _coords(X), _coords(Y)
    w = _complex128(wu)
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).ravel())
    out = np.zeros((r.size, 3), dtype=np.complex128)
    lib().orc_dense_rows_grad(_ptr(X), _ptr(Y), Y.shape[0], _ptr(w), int(kernel) & 1, float(k), _ptr(r), r.size,
                              _ptr(out))
    return out


def lagrange_basis_deriv(r1: int, t: float) -> np.ndarray:
    e = np.zeros(r1)
    lib().orc_lagrange_basis_deriv(r1, float(t), _ptr(e))
    return e


def gauss_legendre(n: int):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gauss_legendre(n, _ptr(x), _ptr(w))
    return x, w


def legendre_p(L: int, t: float) -> np.ndarray:
    P = np.zeros(L + 1)
    lib().orc_legendre_p(L, float(t), _ptr(P))
    return P


def sph_hankel1(L: int, z: float) -> np.ndarray:
    h = np.zeros(L + 1, dtype=np.complex128)
    lib().orc_sph_hankel1(L, float(z), _ptr(h))
    return h


def cheb_nodes(r1: int) -> np.ndarray:
    t = np.zeros(r1)
    lib().orc_cheb_nodes(r1, _ptr(t))
    return t


def lagrange_basis(r1: int, t: float) -> np.ndarray:
    e = np.zeros(r1)
    lib().orc_lagrange_basis(r1, float(t), _ptr(e))
    return e


def gegenbauer_rank(k: float, d_l: float, eps: float) -> int:
    return int(lib().orc_gegenbauer_rank(float(k), float(d_l), float(eps)))


def sphere_quadrature(L: int):
    nq = 2 * L * (L + 1)
    s = np.zeros((nq, 3))
    w = np.zeros(nq)
    lib().orc_sphere_quadrature(L, _ptr(s), _ptr(w))
    return s, w


def gegenbauer_diag(L: int, k: float, r0) -> np.ndarray:
    nq = 2 * L * (L + 1)
    D = np.zeros(nq, dtype=np.complex128)
    r = np.ascontiguousarray(np.asarray(r0, dtype=np.float64))
    lib().orc_gegenbauer_diag(L, float(k), _ptr(r), _ptr(D))
    return D


def es_hat(w: int, beta: float, xi: float) -> float:
    """Fourier transform at xi of the grid form's spreading kernel exp(beta (sqrt(1 - (2t/w)^2) - 1)), |t| < w/2."""
    return float(lib().orc_es_hat(int(w), float(beta), float(xi)))


def grid_forward(p: int, w: int, beta: float, h: float, k: float, L: int, y, u) -> np.ndarray:
    """Grid form of the source transform of one box: u~(q) for the level's quadrature (box-relative points y)."""
    y = _coords(y)
    uu = _complex128(u)
    out = np.zeros(2 * L * (L + 1), dtype=np.complex128)
    lib().orc_grid_forward(int(p), int(w), float(beta), float(h), float(k), int(L), _ptr(y), _ptr(uu), y.shape[0],
                           _ptr(out))
    return out


def grid_backward(p: int, w: int, beta: float, h: float, k: float, L: int, vt, x) -> np.ndarray:
    """Grid form of the target transform of one box: v_i = sum_q e^{ik s_q.x_i} vt(q) at box-relative points x."""
    x = _coords(x)
    v = _complex128(vt)
    out = np.zeros(x.shape[0], dtype=np.complex128)
    lib().orc_grid_backward(int(p), int(w), float(beta), float(h), float(k), int(L), _ptr(v), _ptr(x), x.shape[0],
                            _ptr(out))
    return out


def aca(T, tol: float):
    """Adaptive cross approximation with complete pivoting of a square complex matrix: (A, B) with T ~ A B^T and
    |T - A B^T|_F <= tol |T|_F."""
    T = np.ascontiguousarray(np.asarray(T, dtype=np.complex128))
    r = T.shape[0]
    A = np.zeros((r, r), dtype=np.complex128)
    B = np.zeros((r, r), dtype=np.complex128)
    k = lib().orc_aca(r, _ptr(T), float(tol), _ptr(A), _ptr(B))
    # the C side stores column l contiguously: A[l][i] in this buffer is column l of A
    return A[:k].T.copy(), B[:k].T.copy()


class Plan:
    """The oracle's FFM plan: root cubes, two Morton-sorted octrees, descent lists, leaf.

    ``grid`` maps a Gegenbauer level to the (p, w, beta) of its grid-form transforms; other levels use the
    direct sums.  ``aca`` lists the Lagrange levels whose transfer matrices are compressed by ACA at relative
    tolerance ``aca_tol``."""

    def __init__(self, X, Y, kernel: int, k: float, eps: float, n_leaf: int = 64,
                 kappa: float = 0.0, r1: int = 0, max_level: int = 20, grid: dict | None = None,
                 aca=(), aca_tol: float = 0.0, normals=None, adaptive: bool = False, source_normals=None):
        self.X = _coords(X)
        self.Y = self.X if Y is X else _coords(Y)
        self.kernel, self.k, self.eps = int(kernel), float(k), float(eps)
        opt = _Options(int(n_leaf), float(kappa), int(r1), int(max_level))
        for l, (gp, gw, gb) in (grid or {}).items():
            opt.grid_p[int(l)] = int(gp)
            opt.grid_w[int(l)] = int(gw)
            opt.grid_beta[int(l)] = float(gb)
        opt.aca_tol = float(aca_tol)
        for l in aca:
            opt.aca[int(l)] = 1
        opt.adaptive = 1 if adaptive else 0
        if int(kernel) in (LAPLACE_DN, HELMHOLTZ_DN):
            if normals is None:
                raise ValueError("normal-derivative kernels need the target normals")
            self._normals = _coords(normals)
            opt.target_normals = self._normals.ctypes.data
        if int(kernel) in (LAPLACE_DL, HELMHOLTZ_DL):
            if source_normals is None:
                raise ValueError("double-layer kernels need the source normals")
            self._snormals = _coords(source_normals)
            opt.source_normals = self._snormals.ctypes.data
        self._h = lib().orc_plan_create(_ptr(self.X), self.X.shape[0], _ptr(self.Y), self.Y.shape[0],
                                        self.kernel, self.k, self.eps, C.byref(opt))
        if not self._h:
            raise RuntimeError("oracle plan failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_plan_free(h)
            self._h = None

    def apply(self, wu, stride: int = 1) -> np.ndarray:
        """The product: complex128 (n_x,), or (n_x, 3) for the gradient kernels."""
        w = _complex128(wu)
        grad = self.kernel in (LAPLACE_GRAD, HELMHOLTZ_GRAD)
        v = np.zeros((self.X.shape[0], 3) if grad else self.X.shape[0], dtype=np.complex128)
        lib().orc_apply(self._h, _ptr(w), _ptr(v), int(stride))
        return v

    @property
    def leaf(self) -> int:
        return int(lib().orc_leaf(self._h))

    @property
    def d0(self) -> float:
        return float(lib().orc_d0(self._h))

    def corner(self, s: int) -> np.ndarray:
        c = np.zeros(3)
        lib().orc_corner(self._h, s, _ptr(c))
        return c

    def keys(self, s: int) -> np.ndarray:
        n = lib().orc_npoints(self._h, s)
        a = np.zeros(n, dtype=np.uint64)
        lib().orc_keys(self._h, s, _ptr(a))
        return a

    def perm(self, s: int) -> np.ndarray:
        n = lib().orc_npoints(self._h, s)
        a = np.zeros(n, dtype=np.int64)
        lib().orc_perm(self._h, s, _ptr(a))
        return a

    def nbox(self, s: int, l: int) -> int:
        return int(lib().orc_nbox(self._h, s, l))

    def box_start(self, s: int, l: int) -> np.ndarray:
        a = np.zeros(self.nbox(s, l) + 1, dtype=np.int64)
        lib().orc_box_start(self._h, s, l, _ptr(a))
        return a

    def box_ijk(self, s: int, l: int) -> np.ndarray:
        a = np.zeros((self.nbox(s, l), 3), dtype=np.int32)
        lib().orc_box_ijk(self._h, s, l, _ptr(a))
        return a

    def box_centre(self, s: int, l: int) -> np.ndarray:
        a = np.zeros((self.nbox(s, l), 3))
        lib().orc_box_centre(self._h, s, l, _ptr(a))
        return a

    def far(self, l: int):
        n = lib().orc_nfar(self._h, l)
        t = np.zeros(n, dtype=np.int64)
        s = np.zeros(n, dtype=np.int64)
        o = np.zeros((n, 3), dtype=np.int32)
        if n:
            lib().orc_far(self._h, l, _ptr(t), _ptr(s), _ptr(o))
        return t, s, o

    def near(self, l: int):
        n = lib().orc_nnear(self._h, l)
        t = np.zeros(n, dtype=np.int64)
        s = np.zeros(n, dtype=np.int64)
        if n:
            lib().orc_near(self._h, l, _ptr(t), _ptr(s))
        return t, s

    def early(self, l: int):
        """Near pairs of level l that the per-pair leaf rule sums densely at that level: (t, s) sorted."""
        n = lib().orc_nearly(self._h, l)
        t = np.zeros(n, dtype=np.int64)
        s = np.zeros(n, dtype=np.int64)
        if n:
            lib().orc_early(self._h, l, _ptr(t), _ptr(s))
        return t, s

    def method(self, l: int) -> int:
        return int(lib().orc_level_method(self._h, l))

    def order(self, l: int) -> int:
        return int(lib().orc_level_order(self._h, l))

    def aca_ranks(self, l: int, tol: float) -> dict:
        """ACA rank of every translation class of Lagrange level l: {(ox, oy, oz): rank}."""
        off = np.zeros((400, 3), dtype=np.int32)
        ranks = np.zeros(400, dtype=np.int32)
        n = lib().orc_aca_ranks(self._h, l, float(tol), _ptr(off), _ptr(ranks))
        return {tuple(int(x) for x in off[c]): int(ranks[c]) for c in range(n)}
