"""The gradient at the target, grad_x G(x - y), three components per target (FFM_LAPLACE_GRAD,
FFM_HELMHOLTZ_GRAD): the vector kernels of the integral operators of Sec. 4.2.2, on the GPU through the C ABI.

A gradient plan shares the source transforms and transfers among its components; its target side runs once per
axis c: at Gegenbauer levels the plain target transform (direct, ring or grid form) of ik s_c v~, at Lagrange
levels and in the near field those of the normal derivative with n = e_c, into three output planes gathered to
v[i][c].  Element-wise against the oracle's gradient FFM with identical parameters, grid-form levels included
(FP32_RTOL), within eps of FP64 dense rows, bitwise repeatable; n . v against the GPU's normal-derivative product
(direct forms; within 2 eps); inside a batch, through the server and the no-allocation apply (each bitwise the
plan's own apply); shapes and the output check.
"""
import numpy as np
import pytest

import ffm_workloads as W
from gpu_common import FP32_RTOL, compare_trees, gpu_apply, oracle_like, rel

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("kernel,k,eps,tf", [(6, 0.0, 1e-3, "auto"), (6, 0.0, 1e-4, "auto"), (7, 9.0, 1e-3, "auto"),
                                             (7, 45.0, 1e-3, "auto"), (7, 20.0, 1e-4, "auto"), (7, 45.0, 1e-3, "grid"),
                                             (7, 60.0, 1e-4, "grid")])
def test_grad_matches_oracle_and_dense(orc, kernel, k, eps, tf):
    import paper_1909_05600_amd as ffm
    rng = np.random.default_rng(int(k) + 31)
    Y = W.sphere_points(20000, rng)
    X = W.sphere_points(15000, rng) * 0.985
    wu = ((rng.standard_normal(20000) + 1j * rng.standard_normal(20000)) / 20000).astype(np.complex64)
    print("grad kernel %d k=%g eps=%g transforms %s" % (kernel, k, eps, tf), flush=True)
    gp = ffm.Plan(_dev(X), _dev(Y), kernel, k, eps, transforms=tf)
    st = gp.stats()
    op = oracle_like(orc, gp, X, Y, kernel, k, eps)
    compare_trees(gp, op)
    v = gpu_apply(gp, wu)
    assert v.shape == (15000, 3)
    vo = op.apply(wu)
    rows = np.arange(0, 15000, 29)
    d = orc.dense_rows_grad(X, Y, wu, kernel - 6, k, rows)
    print("grad kernel %d k=%g eps=%g: methods %s forms %s: vs oracle %.3e, vs dense %.3e (oracle %.3e)"
          % (kernel, k, eps, st["method"][:st["leaf"] + 1], st["tform"][:st["leaf"] + 1], rel(v, vo),
             rel(v[rows], d), rel(vo[rows], d)))
    if tf == "grid":
        assert 3 in st["tform"], st["tform"]
    assert rel(v, vo) < FP32_RTOL
    assert rel(v[rows], d) <= eps
    assert np.array_equal(v, gpu_apply(gp, wu))
    # n . grad against the normal-derivative product with the same normals
    N = W.sphere_points(15000, rng)
    dn = gpu_apply(ffm.Plan(_dev(X), _dev(Y), kernel - 4, k, eps, normals=_dev(N)), wu)
    comb = (v * N).sum(axis=1)
    print("n . grad against the normal-derivative plan: %.3e" % rel(comb, dn))
    assert rel(comb, dn) < 2 * eps


def test_grad_batch_server_and_static():
    """One set (the self term excluded) at sizes the static workspace holds: a batch mixing the gradient plan with
    a potential plan, the server and the no-allocation apply each give bitwise the plan's own apply."""
    import torch
    import paper_1909_05600_amd as ffm
    rng = np.random.default_rng(4)
    X = W.sphere_points(12000, rng)
    wu = ((rng.standard_normal(12000) + 1j * rng.standard_normal(12000)) / 12000).astype(np.complex64)
    Xd = _dev(X)
    gp = ffm.Plan(Xd, Xd, ffm.FFM_HELMHOLTZ_GRAD, 15.0, 1e-3)
    v = gpu_apply(gp, wu)
    other = ffm.Plan(Xd, Xd, ffm.FFM_HELMHOLTZ, 15.0, 1e-3)
    ref_other = gpu_apply(other, wu)
    w = _dev(wu)
    print("grad batch", flush=True)
    b = ffm.Batch([gp, other], graph=True)
    outs = b.apply([w, w])
    torch.cuda.synchronize()
    assert tuple(outs[0].shape) == (12000, 3)
    assert np.array_equal(outs[0].cpu().numpy().astype(np.complex128), v)
    assert np.array_equal(outs[1].cpu().numpy().astype(np.complex128), ref_other)
    b.destroy()
    print("grad server", flush=True)
    srv = ffm.Server(slots=2)
    t, out = srv.submit(gp, w)
    srv.wait(t)
    assert np.array_equal(out.cpu().numpy().astype(np.complex128), v)
    srv.destroy()
    print("grad static", flush=True)
    o = gp.apply_static(w)
    torch.cuda.synchronize()
    assert np.array_equal(o.cpu().numpy().astype(np.complex128), v)
    with pytest.raises(ValueError):
        gp.apply(w, out=torch.empty(12000, dtype=torch.complex64, device="cuda"))
    gp.destroy()
    other.destroy()
