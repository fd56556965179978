"""ACA of the Lagrange transfer matrices on the GPU (Sec. 2.2.2, eq. ffmACAmatvec: T ~ A B^T, applied as
A (B^T u~) in one kernel with both products on MFMA; reading R21: complete pivoting, tolerance eps / 4, FP64 on
the host at plan time).

Element-wise against the oracle FFM with identical parameters (its own ACA at the same levels): the rank of
every translation class equal to the oracle's, and v within FP32_RTOL; within eps of FP64 dense rows; close to
the GPU product with full transfer matrices; the planner's automatic choice and both forcing flags.
"""
import numpy as np
import pytest

import ffm_workloads as W
from gpu_common import FP32_RTOL, gpu_apply, gpu_plan, oracle_like, rel

pytestmark = pytest.mark.gpu


def _check_ranks(gp, op, levels):
    import paper_1909_05600_amd as ffm
    for l in levels:
        mine = {tuple(int(x) for x in row[:3]): int(row[3]) for row in gp.export(ffm.FFM_EXPORT_ACA_RANK, 0, l)}
        theirs = op.aca_ranks(l, op.eps / 4)
        assert mine == theirs, l


@pytest.mark.parametrize("kernel,k,eps,n", [(0, 0.0, 1e-4, 20000), (1, 9.0, 1e-3, 20000), (1, 20.0, 1e-4, 30000)])
def test_aca_matches_oracle(orc, kernel, k, eps, n):
    rng = np.random.default_rng(40 + n % 7)
    X = W.sphere_points(n, rng)
    wu = ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / n).astype(np.complex64)
    gp = gpu_plan(X, X, kernel, k, eps)
    st = gp.stats()
    lev = [l for l in range(1, st["leaf"] + 1) if st["aca"][l]]
    assert lev, (st["method"], st["order"], st["aca_rank"])
    op = oracle_like(orc, gp, X, X, kernel, k, eps)
    _check_ranks(gp, op, lev)
    v = gpu_apply(gp, wu)
    vo = op.apply(wu)
    vf = gpu_apply(gpu_plan(X, X, kernel, k, eps, aca="off"), wu)
    rows = np.arange(0, n, 37)
    d = orc.dense_rows(X, X, wu, kernel, k, rows)
    print("kernel %d k=%g eps=%g: ACA levels %s (mean ranks %s of r = %s): vs oracle %.3e, vs dense %.3e, "
          "vs full-T GPU %.3e" % (kernel, k, eps, lev, [round(st["aca_rank"][l], 1) for l in lev],
                                  [st["order"][l] ** 3 for l in lev], rel(v, vo), rel(v[rows], d), rel(v, vf)))
    assert rel(v, vo) < FP32_RTOL
    assert rel(v[rows], d) <= eps
    assert rel(v, vf) <= eps / 2
    assert np.array_equal(v, gpu_apply(gp, wu))


def test_aca_flags(orc):
    """FFM_FLAG_ACA forces ACA at FP32 Lagrange levels with four nodes per axis (r = 64, where the planner keeps
    T); FFM_FLAG_NO_ACA keeps T everywhere; both flags together are refused; mixed precision keeps FP16 T."""
    import paper_1909_05600_amd as ffm
    w = W.laplace_sphere(8192, seed=7)
    auto = gpu_plan(w.X, w.X, 0, 0.0, w.eps)
    assert not any(auto.stats()["aca"])
    forced = gpu_plan(w.X, w.X, 0, 0.0, w.eps, aca="on")
    lev = [l for l in range(1, forced.stats()["leaf"] + 1) if forced.stats()["aca"][l]]
    assert lev
    op = oracle_like(orc, forced, w.X, w.X, 0, 0.0, w.eps)
    _check_ranks(forced, op, lev)
    v = gpu_apply(forced, w.wu)
    assert rel(v, op.apply(w.wu)) < FP32_RTOL
    assert rel(v, gpu_apply(auto, w.wu)) <= w.eps / 2
    off = gpu_plan(w.X, w.X, 0, 0.0, 1e-4, aca="off")
    assert not any(off.stats()["aca"])
    mixed = gpu_plan(w.X, w.X, 0, 0.0, w.eps, aca="on", precision=1)
    assert not any(mixed.stats()["aca"]) and any(mixed.stats()["prec"])
    import ctypes as C
    h = C.c_void_p()
    Xd = __import__("torch").from_numpy(w.X).cuda()
    bad = ffm.Options(0, 0, 0.0, 0, 0, ffm.FFM_FLAG_ACA | ffm.FFM_FLAG_NO_ACA)
    assert ffm.lib().ffm_plan(Xd.data_ptr(), w.n, Xd.data_ptr(), w.n, 0, 0.0, 1e-3, C.byref(bad), None,
                              C.byref(h)) == -1


def test_aca_in_a_batch():
    """A batch mixing ACA and full-T levels gives each instance bitwise its own apply."""
    import torch
    import paper_1909_05600_amd as ffm
    rng = np.random.default_rng(3)
    plans, wus, refs = [], [], []
    for n, kern, k, eps, aca in ((9000, 1, 15.0, 1e-3, "auto"), (7000, 0, 0.0, 1e-4, "auto"),
                                 (6000, 0, 0.0, 1e-3, "off"), (5000, 1, 6.0, 1e-3, "on")):
        X = W.sphere_points(n, rng)
        wu = ((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / n).astype(np.complex64)
        p = gpu_plan(X, X, kern, k, eps, aca=aca)
        plans.append(p)
        wus.append(torch.from_numpy(wu).cuda())
        refs.append(gpu_apply(p, wu))
    assert sum(any(p.stats()["aca"]) for p in plans) >= 2
    b = ffm.Batch(plans, graph=True)
    outs = b.apply(wus)
    torch.cuda.synchronize()
    for o, r in zip(outs, refs):
        assert np.array_equal(o.cpu().numpy().astype(np.complex128), r)
    b.destroy()
