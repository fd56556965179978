"""ffm_apply_static: the apply over the library's static device workspace, for callers that cannot allocate.

Checked through the C ABI against ffm_apply on the same plans (same kernels and work items over another
workspace: equal bitwise, and within FP32_RTOL of the FP64 oracle with identical parameters), on two calls
in a row, the second on a smaller plan, then the first again (the workspace keeps the previous call's
contents; the kernels clear what must start at zero).  A plan whose workspace exceeds the static size is
rejected with a message naming both sizes.  Not in the paper.
"""
import ctypes as C

import numpy as np
import pytest

import ffm_workloads as W
from gpu_common import FP32_RTOL, gpu_plan, oracle_like, rel

pytestmark = pytest.mark.gpu


def _static(p, wu_np):
    import torch
    import paper_1909_05600_amd as ffm
    wu = torch.from_numpy(np.ascontiguousarray(wu_np)).cuda()
    out = torch.full((p.n_x,), complex(7.0, -3.0), dtype=torch.complex64, device="cuda")   # stale contents
    torch.cuda.synchronize()
    rc = ffm.lib().ffm_apply_static(p._h, wu.data_ptr(), ffm._dtype_code(wu), out.data_ptr(), None)
    assert rc == 0, ffm.lib().ffm_last_error()
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.complex128)


def _apply(p, wu_np):
    import torch
    wu = torch.from_numpy(np.ascontiguousarray(wu_np)).cuda()
    v = p.apply(wu)
    torch.cuda.synchronize()
    return v.cpu().numpy().astype(np.complex128)


def test_static_apply_equals_apply(orc):
    import paper_1909_05600_amd as ffm
    big = W.helmholtz_sphere(40000, seed=21, k=60.0, n_rows=64)        # grid-form and direct levels
    small = W.laplace_sphere(6000, seed=22)
    pb = gpu_plan(big.X, big.X, 1, big.k, big.eps)
    ps = gpu_plan(small.X, small.X, 0, 0.0, small.eps)
    for p in (pb, ps):
        print("workspace %d bytes (static %d)" % (p.workspace_bytes(), ffm.STATIC_WORKSPACE_BYTES))
        assert p.workspace_bytes() <= ffm.STATIC_WORKSPACE_BYTES
    ref_b, ref_s = _apply(pb, big.wu), _apply(ps, small.wu)
    got_b = _static(pb, big.wu)
    got_s = _static(ps, small.wu)                                   # second call: a smaller input
    again_b = _static(pb, big.wu)                                   # and the larger one again
    assert np.array_equal(got_b, ref_b)
    assert np.array_equal(got_s, ref_s)
    assert np.array_equal(again_b, ref_b)
    assert rel(got_b, oracle_like(orc, pb, big.X, big.X, 1, big.k, big.eps).apply(big.wu)) < FP32_RTOL
    assert rel(got_s, oracle_like(orc, ps, small.X, small.X, 0, 0.0, small.eps).apply(small.wu)) < FP32_RTOL
    # retiled plans rebuild their static descriptors with their launches
    pb.set_tiles(2, 1)
    assert np.array_equal(_static(pb, big.wu), _apply(pb, big.wu))
    pb.destroy()
    ps.destroy()


def test_static_apply_rejects_plans_that_do_not_fit():
    import torch
    import paper_1909_05600_amd as ffm
    w = W.helmholtz_sphere(1 << 20, seed=2, n_rows=16)
    p = gpu_plan(w.X, w.X, 1, w.k, w.eps)
    assert p.workspace_bytes() > ffm.STATIC_WORKSPACE_BYTES
    wu = torch.from_numpy(w.wu).cuda()
    with pytest.raises(ffm.FFMError) as e:
        p.apply_static(wu)
    assert e.value.code == -1 and "exceeds the static workspace" in str(e.value)
    # an empty set: zeros, no workspace needed
    X = W.sphere_points(50, np.random.default_rng(1))
    pe = gpu_plan(X, np.zeros((0, 3)), 0, 0.0, 1e-3)
    out = pe.apply_static(torch.zeros(0, dtype=torch.complex64, device="cuda"),
                          out=torch.ones(50, dtype=torch.complex64, device="cuda"))
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    p.destroy()
    pe.destroy()
