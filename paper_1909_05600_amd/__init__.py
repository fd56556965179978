"""Python binding of the gfx950 Fast Free Memory library (libffm.so).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI declared in ``include/ffm.h``.  PyTorch provides device
memory and streams.  Importing this package does not build anything; a
missing library raises at first use, loudly (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libffm.so")

FFM_LAPLACE = 0
FFM_HELMHOLTZ = 1
FFM_LAPLACE_DN = 2          # normal derivative at the target (adjoint double-layer kernel)
FFM_HELMHOLTZ_DN = 3
FFM_LAPLACE_DL = 4          # normal derivative at the source (double-layer kernel)
FFM_HELMHOLTZ_DL = 5
FFM_LAPLACE_GRAD = 6        # gradient at the target (three components per target)
FFM_HELMHOLTZ_GRAD = 7
FFM_C64, FFM_F32, FFM_F64, FFM_C128 = 0, 1, 2, 3
FFM_PREC_FP32, FFM_PREC_MIXED = 0, 1
FFM_EXPORT_KEYS, FFM_EXPORT_PERM, FFM_EXPORT_BOX_START, FFM_EXPORT_BOX_IJK = 0, 1, 2, 3
FFM_EXPORT_BOX_CTR, FFM_EXPORT_FAR, FFM_EXPORT_NEAR, FFM_EXPORT_ACA_RANK, FFM_EXPORT_EARLY = 4, 5, 6, 7, 8
MAX_LEVELS = 21

STATUS = {0: "FFM_OK", -1: "FFM_EINVAL", -2: "FFM_ENOMEM", -3: "FFM_EDEVICE", -4: "FFM_EBUSY", -5: "FFM_EINTERNAL"}

# every symbol the C ABI exports (include/ffm.h)
EXPORTED = ["ffm_plan", "ffm_apply", "ffm_destroy", "ffm_last_error", "ffm_version", "ffm_plan_stats",
            "ffm_plan_export", "ffm_plan_timing", "ffm_plan_bytes", "ffm_workspace_bytes",
            "ffm_plan_set_tiles", "ffm_plan_get_tiles", "ffm_batch_create", "ffm_batch_apply", "ffm_batch_info",
            "ffm_batch_destroy", "ffm_server_create", "ffm_server_submit", "ffm_server_wait", "ffm_server_poll",
            "ffm_server_stats", "ffm_server_destroy", "ffm_plan_launch_timing", "ffm_kernel_name",
            "ffm_apply_batched", "ffm_apply_static", "ffm_device_bytes_live"]
STATIC_WORKSPACE_BYTES = 128 << 20
FFM_FLAG_TIMING = 1
FFM_FLAG_DIRECT_TRANSFORMS = 2
FFM_FLAG_GRID_TRANSFORMS = 4
FFM_FLAG_NO_ACA = 8
FFM_FLAG_ACA = 16
FFM_FLAG_ADAPTIVE_LEAVES = 32
FFM_BATCH_GRAPH = 1
FFM_BATCH_AUTOTUNE = 2
TIMING_SLOTS = 64


class FFMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(code, str(code)), msg))
        self.code = code


class Options(C.Structure):
    _fields_ = [("n_leaf", C.c_int32), ("precision", C.c_int32), ("kd_switch", C.c_double),
                ("r1_override", C.c_int32), ("max_level", C.c_int32), ("flags", C.c_uint32),
                ("target_normals", C.c_void_p), ("source_normals", C.c_void_p)]


_L = MAX_LEVELS


class Stats(C.Structure):
    _fields_ = [("leaf", C.c_int32), ("same_set", C.c_int32), ("d0", C.c_double),
                ("corner_x", C.c_double * 3), ("corner_y", C.c_double * 3),
                ("nbox_x", C.c_int64 * _L), ("nbox_y", C.c_int64 * _L), ("nfar", C.c_int64 * _L),
                ("nnear", C.c_int64 * _L), ("method", C.c_int32 * _L), ("order", C.c_int32 * _L),
                ("tform", C.c_int32 * _L), ("prec", C.c_int32 * _L), ("phase64", C.c_int32 * _L),
                ("nclass", C.c_int32 * _L), ("nq", C.c_int64 * _L), ("fwd_points", C.c_double * _L),
                ("bwd_points", C.c_double * _L), ("transform_terms", C.c_double),
                ("transfer_macs", C.c_double), ("near_pairs", C.c_double), ("plan_bytes", C.c_double),
                ("workspace_bytes", C.c_double), ("grid_nodes", C.c_int32 * _L), ("fwd_boxes", C.c_int64 * _L),
                ("bwd_boxes", C.c_int64 * _L), ("grid_width", C.c_int32 * _L), ("grid_beta", C.c_double * _L),
                ("grid_alias", C.c_double * _L), ("aca", C.c_int32 * _L), ("aca_rank", C.c_double * _L),
                ("nearly", C.c_int64 * _L)]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class Tiles(C.Structure):
    _fields_ = [("ring_g", C.c_int32), ("bwd_pt", C.c_int32)]


class BatchInfo(C.Structure):
    _fields_ = [("n", C.c_int32), ("launches", C.c_int32), ("graph", C.c_int32), ("tuned", C.c_int32),
                ("tiles", Tiles), ("tuned_ms", C.c_float * 4), ("work_items", C.c_int64)]


class ServerOptions(C.Structure):
    _fields_ = [("slots", C.c_int32), ("reserved", C.c_int32), ("budget_bytes", C.c_double)]


class Launch(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("variant_a", C.c_int32), ("variant_b", C.c_int32), ("level", C.c_int32),
                ("blocks", C.c_int64), ("ms", C.c_float), ("reserved", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("slots", C.c_int32), ("running", C.c_int32), ("peak_running", C.c_int32),
                ("reserved", C.c_int32), ("completed", C.c_int64), ("failed", C.c_int64), ("queued", C.c_int64),
                ("budget_bytes", C.c_double), ("in_use_bytes", C.c_double), ("peak_in_use_bytes", C.c_double),
                ("points", C.c_double), ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("max_ms", C.c_double)]


_lib = None


def lib():
    """Load libffm.so (built by paper_1909_05600_amd.build); raise if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libffm.so is not built: run paper_1909_05600_amd.build.build() "
                               "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        P, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        sig = {
            "ffm_plan": (C.c_int, [P, i64, P, i64, C.c_int, dbl, dbl, P, P, P]),
            "ffm_apply": (C.c_int, [P, P, C.c_int, P, P]),
            "ffm_destroy": (C.c_int, [P]),
            "ffm_last_error": (C.c_char_p, []),
            "ffm_version": (C.c_char_p, []),
            "ffm_plan_stats": (C.c_int, [P, P]),
            "ffm_plan_export": (C.c_int, [P, i32, i32, i32, P, P]),
            "ffm_plan_timing": (C.c_int, [P, P, i32]),
            "ffm_plan_bytes": (C.c_size_t, [P]),
            "ffm_workspace_bytes": (C.c_size_t, [P]),
            "ffm_device_bytes_live": (C.c_size_t, []),
            "ffm_plan_set_tiles": (C.c_int, [P, P, P]),
            "ffm_plan_get_tiles": (C.c_int, [P, P]),
            "ffm_batch_create": (C.c_int, [P, i32, C.c_uint32, C.c_char_p, P, P]),
            "ffm_batch_apply": (C.c_int, [P, P, P, P, P]),
            "ffm_batch_info": (C.c_int, [P, P]),
            "ffm_batch_destroy": (C.c_int, [P]),
            "ffm_server_create": (C.c_int, [P, P]),
            "ffm_server_submit": (C.c_int, [P, P, P, C.c_int, P, P, P]),
            "ffm_apply_batched": (C.c_int, [P, P, P, i32, P]),
            "ffm_apply_static": (C.c_int, [P, P, C.c_int, P, P]),
            "ffm_server_wait": (C.c_int, [P, i64, P]),
            "ffm_server_poll": (C.c_int, [P, i64, P]),
            "ffm_server_stats": (C.c_int, [P, P]),
            "ffm_server_destroy": (C.c_int, [P]),
            "ffm_plan_launch_timing": (C.c_int, [P, P, i32, P]),
            "ffm_kernel_name": (i32, [i32, i32, i32, C.c_char_p, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise FFMError(rc, lib().ffm_last_error().decode(errors="replace"))


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


# ---------------------------------------------------------------- thin C-ABI mirrors
def ffm_plan(X_ptr: int, n_x: int, Y_ptr: int, n_y: int, kernel: int, k: float, eps: float,
             opts: Options | None = None, stream: int = 0) -> int:
    h = C.c_void_p()
    _check(lib().ffm_plan(X_ptr, n_x, Y_ptr, n_y, kernel, k, eps, C.byref(opts) if opts else None,
                          stream, C.byref(h)))
    return h.value


def ffm_apply(plan: int, wu_ptr: int, in_dtype: int, v_ptr: int, stream: int = 0) -> None:
    _check(lib().ffm_apply(plan, wu_ptr, in_dtype, v_ptr, stream))


def ffm_destroy(plan: int) -> None:
    _check(lib().ffm_destroy(plan))


def apply_batched(plans, wus, outs=None, stream=None):
    """v[i] = FFM_i(wu[i]) for distinct plans in one pass of merged launches (ffm_apply_batched); complex64
    inputs.  Returns the outputs (complex64, each instance's caller order)."""
    import torch
    n = len(plans)
    if len(wus) != n or n == 0:
        raise ValueError("one input per plan, at least one plan")
    wus = [w.contiguous() for w in wus]
    for p, w in zip(plans, wus):
        if w.dtype != torch.complex64 or w.shape[0] != p.n_y or not w.is_cuda:
            raise ValueError("wu[i] must be a complex64 CUDA tensor of length n_y of plan i")
    outs = [_out(p, None, "outs[i]") for p in plans] if outs is None else \
        [_out(p, o, "outs[i]") for p, o in zip(plans, outs)]
    hp = (C.c_void_p * n)(*[p._h for p in plans])
    wp = (C.c_void_p * n)(*[w.data_ptr() for w in wus])
    vp = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    _check(lib().ffm_apply_batched(hp, wp, vp, n, _stream(stream)))
    return outs


def ffm_version() -> str:
    return lib().ffm_version().decode()


# ---------------------------------------------------------------- torch-facing helper
_DTYPES = None


def _dtype_code(t) -> int:
    import torch
    global _DTYPES
    if _DTYPES is None:
        _DTYPES = {torch.complex64: FFM_C64, torch.float32: FFM_F32, torch.float64: FFM_F64,
                   torch.complex128: FFM_C128}
    if t.dtype not in _DTYPES:
        raise TypeError("wu must be complex64, complex128, float32 or float64")
    return _DTYPES[t.dtype]


def device_bytes_live() -> int:
    """Device bytes the library holds in live allocations (its cache of freed blocks excluded)."""
    return int(lib().ffm_device_bytes_live())


def kernel_name(kernel: int, variant_a: int = 0, variant_b: int = 0) -> str:
    """Symbol of a launch's kernel as profilers print it (ffm_kernel_name)."""
    buf = C.create_string_buffer(96)
    n = lib().ffm_kernel_name(kernel, variant_a, variant_b, buf, 96)
    if n < 0:
        raise FFMError(-1, "unknown kernel %d" % kernel)
    return buf.value.decode()


def _out(plan, o, what="out"):
    """The output tensor of a product of ``plan`` (allocated when o is None): complex64 (n_x,), or (n_x, 3)
    for the gradient kernels, contiguous on the plan's device."""
    import torch
    if o is None:
        return torch.empty(plan.out_shape, dtype=torch.complex64, device=plan.device)
    if o.dtype != torch.complex64 or o.numel() != plan.n_x * plan.ncomp or not o.is_contiguous():
        raise ValueError("%s must be a contiguous complex64 tensor of n_x (x 3 for gradient plans) elements" % what)
    return o


class Plan:
    """An FFM plan over device coordinates X (targets) and Y (sources).

    ``Plan(X, Y, kernel, k, eps)`` with X, Y FP64 CUDA tensors of shape (n, 3);
    pass the same tensor object twice for one set.  ``apply(wu)`` returns v as
    complex64 on the device, in the caller's order.
    """

    def __init__(self, X, Y, kernel: int, k: float, eps: float, n_leaf: int = 0, precision: int = 0,
                 kd_switch: float = 0.0, r1_override: int = 0, max_level: int = 0, timing: bool = False,
                 transforms: str = "auto", aca: str = "auto", normals=None, adaptive: bool = False, stream=None,
                 source_normals=None):
        import torch
        same = Y is X
        X = X.detach().contiguous()
        if X.dtype != torch.float64 or X.dim() != 2 or X.shape[1] != 3 or not X.is_cuda:
            raise TypeError("X must be a CUDA float64 tensor of shape (n, 3)")
        if same:
            Y = X
        else:
            Y = Y.detach().contiguous()
            if Y.dtype != torch.float64 or Y.dim() != 2 or Y.shape[1] != 3 or not Y.is_cuda:
                raise TypeError("Y must be a CUDA float64 tensor of shape (n, 3)")
        self.n_x, self.n_y = int(X.shape[0]), int(Y.shape[0])
        self.kernel, self.k, self.eps = int(kernel), float(k), float(eps)
        self.ncomp = 3 if self.kernel in (FFM_LAPLACE_GRAD, FFM_HELMHOLTZ_GRAD) else 1
        self.out_shape = (self.n_x, 3) if self.ncomp == 3 else (self.n_x,)
        self.device = X.device
        flags = (FFM_FLAG_TIMING if timing else 0) | {"auto": 0, "direct": FFM_FLAG_DIRECT_TRANSFORMS,
                                                      "grid": FFM_FLAG_GRID_TRANSFORMS}[transforms] | \
            {"auto": 0, "off": FFM_FLAG_NO_ACA, "on": FFM_FLAG_ACA}[aca] | (FFM_FLAG_ADAPTIVE_LEAVES if adaptive else 0)
        opts = Options(int(n_leaf), int(precision), float(kd_switch), int(r1_override), int(max_level), flags)
        if normals is not None:
            normals = normals.detach().contiguous()
            if normals.dtype != torch.float64 or normals.shape != X.shape or not normals.is_cuda:
                raise TypeError("normals must be a CUDA float64 tensor shaped like X")
            opts.target_normals = normals.data_ptr()
        if source_normals is not None:
            source_normals = source_normals.detach().contiguous()
            if source_normals.dtype != torch.float64 or source_normals.shape != Y.shape or not source_normals.is_cuda:
                raise TypeError("source_normals must be a CUDA float64 tensor shaped like Y")
            opts.source_normals = source_normals.data_ptr()
        self._h = None
        with torch.cuda.device(self.device):
            self._h = ffm_plan(X.data_ptr(), self.n_x, Y.data_ptr(), self.n_y, self.kernel, self.k, self.eps,
                               opts, _stream(stream))

    def apply(self, wu, out=None, stream=None):
        import torch
        if wu.shape[0] != self.n_y or not wu.is_cuda:
            raise ValueError("wu must be a CUDA tensor of length n_y")
        wu = wu.contiguous()
        out = _out(self, out)
        ffm_apply(self._h, wu.data_ptr(), _dtype_code(wu), out.data_ptr(), _stream(stream))
        return out

    def apply_static(self, wu, out=None, stream=None):
        """apply() over the library's static device workspace (ffm_apply_static): no allocation inside the call
        (pass ``out`` to keep the Python side allocation-free too).  Plans whose workspace exceeds
        STATIC_WORKSPACE_BYTES are rejected; calls that overlap on one device race."""
        import torch
        if wu.shape[0] != self.n_y or not wu.is_cuda or not wu.is_contiguous():
            raise ValueError("wu must be a contiguous CUDA tensor of length n_y")
        out = _out(self, out)
        _check(lib().ffm_apply_static(self._h, wu.data_ptr(), _dtype_code(wu), out.data_ptr(), _stream(stream)))
        return out

    def stats(self) -> dict:
        s = Stats()
        _check(lib().ffm_plan_stats(self._h, C.byref(s)))
        return s.as_dict()

    def export(self, what: int, set_: int = 0, level: int = 0):
        import numpy as np
        cnt = C.c_int64()
        _check(lib().ffm_plan_export(self._h, what, set_, level, None, C.byref(cnt)))
        dt = {FFM_EXPORT_KEYS: np.uint64, FFM_EXPORT_BOX_IJK: np.int32, FFM_EXPORT_BOX_CTR: np.float64}.get(
            what, np.int64)
        a = np.zeros(cnt.value, dtype=dt)
        if cnt.value:
            _check(lib().ffm_plan_export(self._h, what, set_, level, a.ctypes.data_as(C.c_void_p),
                                         C.byref(cnt)))
        if what in (FFM_EXPORT_BOX_IJK, FFM_EXPORT_BOX_CTR):
            a = a.reshape(-1, 3)
        elif what == FFM_EXPORT_FAR:
            a = a.reshape(-1, 5)
        elif what in (FFM_EXPORT_NEAR, FFM_EXPORT_EARLY):
            a = a.reshape(-1, 2)
        elif what == FFM_EXPORT_ACA_RANK:
            a = a.reshape(-1, 4)
        return a

    def timing(self) -> list:
        """Per-phase milliseconds of the last apply (plans made with timing=True)."""
        buf = (C.c_float * TIMING_SLOTS)()
        _check(lib().ffm_plan_timing(self._h, buf, TIMING_SLOTS))
        return list(buf)

    def launch_timing(self) -> list:
        """The kernel launches of the last apply (plans made with timing=True), in order: dicts with the kernel's
        symbol, its level, thread blocks and HIP-event milliseconds."""
        n = C.c_int32(0)
        _check(lib().ffm_plan_launch_timing(self._h, None, 0, C.byref(n)))
        buf = (Launch * max(n.value, 1))()
        _check(lib().ffm_plan_launch_timing(self._h, buf, n.value, C.byref(n)))
        return [{"kernel": kernel_name(r.kernel, r.variant_a, r.variant_b), "level": r.level, "blocks": r.blocks,
                 "ms": r.ms} for r in buf[:n.value]]

    def set_tiles(self, ring_g: int, bwd_pt: int, stream=None):
        """Rebuild the plane-wave kernels' launches for a tile choice (ring_g in {2, 4}, bwd_pt in {1, 2})."""
        _check(lib().ffm_plan_set_tiles(self._h, C.byref(Tiles(int(ring_g), int(bwd_pt))), _stream(stream)))

    def tiles(self) -> tuple:
        t = Tiles()
        _check(lib().ffm_plan_get_tiles(self._h, C.byref(t)))
        return (t.ring_g, t.bwd_pt)

    def plan_bytes(self) -> int:
        return int(lib().ffm_plan_bytes(self._h))

    def workspace_bytes(self) -> int:
        return int(lib().ffm_workspace_bytes(self._h))

    def destroy(self):
        if self._h:
            ffm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().ffm_destroy(self._h)
                self._h = None
        except Exception:
            pass


class Batch:
    """Many plans applied together: one launch per step kind for all instances (ffm_batch_*).

    ``Batch(plans, graph=True, autotune=False, cache=None)``; ``apply(wus, outs=None)`` returns the list of
    outputs (complex64, each instance's caller order).  The plans stay owned by the caller and must outlive
    the batch (the batch keeps references to them).
    """

    def __init__(self, plans, graph: bool = True, autotune: bool = False, cache: str | None = None, stream=None):
        import torch
        self.plans = list(plans)
        n = len(self.plans)
        arr = (C.c_void_p * n)(*[p._h for p in self.plans])
        flags = (FFM_BATCH_GRAPH if graph else 0) | (FFM_BATCH_AUTOTUNE if autotune else 0)
        h = C.c_void_p()
        self._h = None
        with torch.cuda.device(self.plans[0].device):
            _check(lib().ffm_batch_create(arr, n, flags, cache.encode() if cache else None, _stream(stream),
                                          C.byref(h)))
        self._h = h.value

    def apply(self, wus, outs=None, stream=None):
        import torch
        n = len(self.plans)
        if len(wus) != n:
            raise ValueError("one input per plan")
        wus = [w.contiguous() for w in wus]
        for p, w in zip(self.plans, wus):
            if w.shape[0] != p.n_y or not w.is_cuda:
                raise ValueError("wu[i] must be a CUDA tensor of length n_y of plan i")
        outs = [_out(p, None, "outs[i]") for p in self.plans] if outs is None else \
            [_out(p, o, "outs[i]") for p, o in zip(self.plans, outs)]
        wp = (C.c_void_p * n)(*[w.data_ptr() for w in wus])
        dt = (C.c_int32 * n)(*[_dtype_code(w) for w in wus])
        vp = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        self._keep = (wus, outs)
        _check(lib().ffm_batch_apply(self._h, wp, dt, vp, _stream(stream)))
        return outs

    def info(self) -> dict:
        b = BatchInfo()
        _check(lib().ffm_batch_info(self._h, C.byref(b)))
        return {"n": b.n, "launches": b.launches, "graph": b.graph, "tuned": b.tuned,
                "tiles": (b.tiles.ring_g, b.tiles.bwd_pt), "tuned_ms": list(b.tuned_ms),
                "work_items": b.work_items}

    def destroy(self):
        if self._h:
            _check(lib().ffm_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().ffm_batch_destroy(self._h)
                self._h = None
        except Exception:
            pass


class Server:
    """Resident-plan request loop (ffm_server_*): ``submit(plan, wu, out=None)`` queues one apply and returns
    (ticket, out); ``wait(ticket)`` blocks until it completes and returns its latency in ms."""

    def __init__(self, slots: int = 4, budget_bytes: float = 0.0):
        opts = ServerOptions(int(slots), 0, float(budget_bytes))
        h = C.c_void_p()
        self._h = None
        _check(lib().ffm_server_create(C.byref(opts), C.byref(h)))
        self._h = h.value
        self._live = {}

    def submit(self, plan: Plan, wu, out=None, stream=None):
        """Queue one apply; the request is ordered after the work already enqueued on ``stream`` (default:
        the current stream), which is where wu is expected to be produced."""
        import torch
        if wu.shape[0] != plan.n_y or not wu.is_cuda or not wu.is_contiguous():
            raise ValueError("wu must be a contiguous CUDA tensor of length n_y")
        out = _out(plan, out)
        t = C.c_int64()
        _check(lib().ffm_server_submit(self._h, plan._h, wu.data_ptr(), _dtype_code(wu), out.data_ptr(),
                                       _stream(stream), C.byref(t)))
        self._live[t.value] = (plan, wu, out)     # keep the buffers alive until the request is waited for
        return t.value, out

    def wait(self, ticket: int) -> float:
        lat = C.c_double()
        try:
            _check(lib().ffm_server_wait(self._h, int(ticket), C.byref(lat)))
        finally:
            self._live.pop(int(ticket), None)
        return lat.value

    def poll(self, ticket: int) -> bool:
        d = C.c_int32()
        _check(lib().ffm_server_poll(self._h, int(ticket), C.byref(d)))
        return bool(d.value)

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().ffm_server_stats(self._h, C.byref(s)))
        return {name: getattr(s, name) for name, _ in s._fields_ if name != "reserved"}

    def destroy(self):
        if self._h:
            _check(lib().ffm_server_destroy(self._h))
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().ffm_server_destroy(self._h)
                self._h = None
        except Exception:
            pass
