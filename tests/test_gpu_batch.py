"""Batched application: many plans in one set of merged launches, eager and replayed from a HIP graph.

Every instance of a batch must equal, bitwise, the apply of its own plan with the same tiles (owner-
computes kernels, identical work items); graph replays are checked against the eager batch with other
GPU work and synchronisations between replays; the tile autotuner's choice is cached and reused.
Paper: Sec. 2.2 (the product each instance computes); the batching itself is not in the paper.
"""
import json
import math

import numpy as np
import pytest

import ffm_workloads as W
from gpu_common import FP32_RTOL, gpu_apply, gpu_plan, oracle_like, rel

pytestmark = pytest.mark.gpu


def _mixed_instances():
    """A small mix of every kind of level and kernel variant: cfg4-like instances (sphere, ellipsoid, cube;
    Laplace and Helmholtz), a Helmholtz sphere with ring-pair levels (L >= 64), one with grid-form levels
    (spreading, MFMA plane sums, interpolation), a mixed-precision Laplace
    plan (FP16 MFMA transfers), distinct source and target sets, and plans without sources or targets."""
    import torch
    ws = W.batched_instances(9, seed=4, n_min=2000, n_max=30000)
    specs = [(w.X, w.X, w.kernel, w.k, w.eps, {}, w.wu) for w in ws]
    h = W.helmholtz_sphere(40000, seed=7, k=100.0)
    specs.append((h.X, h.X, 1, h.k, h.eps, {}, h.wu))
    g = W.helmholtz_sphere(30000, seed=10, k=60.0)
    specs.append((g.X, g.X, 1, g.k, g.eps, {"transforms": "grid"}, g.wu))   # grid-form levels
    l = W.laplace_sphere(20000, seed=8)
    specs.append((l.X, l.X, 0, 0.0, l.eps, {"precision": 1}, l.wu.astype(np.complex64)))
    rng = np.random.default_rng(9)
    X = W.sphere_points(7000, rng)
    Y = W.sphere_points(5000, rng) * 0.9 + 0.05
    wu = ((rng.standard_normal(5000) + 1j * rng.standard_normal(5000)) / 5000).astype(np.complex64)
    specs.append((X, Y, 1, 12.0, 1e-3, {}, wu))
    specs.append((X[:300], np.zeros((0, 3)), 0, 0.0, 1e-3, {}, np.zeros(0, np.complex64)))
    specs.append((np.zeros((0, 3)), Y[:200], 1, 3.0, 1e-3, {}, wu[:200]))
    plans, wus = [], []
    for X_, Y_, kern, k, eps, kw, w in specs:
        plans.append(gpu_plan(X_, X_ if Y_ is X_ else Y_, kern, k, eps, **kw))
        wus.append(torch.from_numpy(np.ascontiguousarray(w)).cuda())
    return plans, wus, specs


def _standalone(plans, wus):
    import torch
    outs = [p.apply(w) for p, w in zip(plans, wus)]
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def test_batch_equals_standalone_eager_and_graph():
    import torch
    import paper_1909_05600_amd as ffm
    plans, wus, _ = _mixed_instances()
    ref = _standalone(plans, wus)
    b = ffm.Batch(plans, graph=False)
    info = b.info()
    assert info["n"] == len(plans) and info["graph"] == 0
    outs = b.apply(wus)
    torch.cuda.synchronize()
    for i, (o, r) in enumerate(zip(outs, ref)):
        assert np.array_equal(o.cpu().numpy(), r), i
    b.destroy()

    g = ffm.Batch(plans, graph=True)
    assert g.info()["graph"] == 1
    gen = torch.Generator(device="cuda").manual_seed(11)
    for rep in range(4):
        # new inputs every replay; other GPU work and synchronisations between replays
        wus_r = [w * (1.0 + 0.5 * rep) if w.dtype.is_complex else w for w in wus]
        outs = g.apply(wus_r)
        junk = torch.randn(1 << 20, device="cuda", generator=gen).cumsum(0)
        torch.cuda.synchronize()
        got = [o.cpu().numpy() for o in outs]
        want = _standalone(plans, wus_r)
        for i, (a, r) in enumerate(zip(got, want)):
            assert np.array_equal(a, r), (rep, i)
        del junk
    g.destroy()
    for p in plans:
        p.destroy()


def test_batch_matches_oracle(orc):
    """Direct parity of batched instances with the FP64 oracle FFM (identical parameters) and dense rows."""
    import torch
    import paper_1909_05600_amd as ffm
    plans, wus, specs = _mixed_instances()
    b = ffm.Batch(plans, graph=True)
    outs = b.apply(wus)
    torch.cuda.synchronize()
    for i in (0, 1, 2, 9, 10):          # 10: grid-form levels
        X, Y, kern, k, eps, kw, w = specs[i]
        op = oracle_like(orc, plans[i], X, X if Y is X else Y, kern, k, eps)
        vo = op.apply(w)
        v = outs[i].cpu().numpy().astype(np.complex128)
        rows = np.arange(0, X.shape[0], max(1, X.shape[0] // 256))
        d = orc.dense_rows(X, X if Y is X else Y, w, kern, k, rows)
        print("instance %d (N=%d kernel %d k=%.2f): vs oracle %.3e vs dense %.3e"
              % (i, X.shape[0], kern, k, rel(v, vo), rel(v[rows], d)))
        assert rel(v, vo) < FP32_RTOL
        assert rel(v[rows], d) <= eps
    b.destroy()


def test_tiles_change_only_rounding():
    """Tiles only regroup partial sums (forward point segments, target-transform ring parts): results agree
    to rounding, and an apply is bitwise reproducible for fixed tiles."""
    import torch
    w = W.helmholtz_sphere(40000, seed=7, k=100.0)
    p = gpu_plan(w.X, w.X, 1, w.k, w.eps)
    assert max(p.stats()["order"]) >= 64
    assert p.tiles() == (4, 2)
    v42 = gpu_apply(p, w.wu)
    p.set_tiles(4, 1)
    v41 = gpu_apply(p, w.wu)
    p.set_tiles(2, 2)
    v22 = gpu_apply(p, w.wu)
    assert p.tiles() == (2, 2)
    assert np.array_equal(v22, gpu_apply(p, w.wu))
    assert rel(v41, v42) < 1e-5
    assert rel(v22, v42) < 1e-5


def test_autotune_and_cache(tmp_path):
    import torch
    import paper_1909_05600_amd as ffm
    plans, wus, _ = _mixed_instances()
    cache = str(tmp_path / "tiles.json")
    b = ffm.Batch(plans, graph=True, autotune=True, cache=cache)
    info = b.info()
    assert info["tuned"] == 1 and min(info["tuned_ms"]) > 0
    c = (0 if info["tiles"][0] == 4 else 2) + (0 if info["tiles"][1] == 2 else 1)
    assert info["tuned_ms"][c] == min(info["tuned_ms"])
    data = json.load(open(cache))
    assert len(data) == 1
    (ent,) = data.values()
    assert (ent["ring_g"], ent["bwd_pt"]) == info["tiles"]
    outs = b.apply(wus)
    torch.cuda.synchronize()
    got = [o.cpu().numpy() for o in outs]
    b.destroy()
    # the plans keep the tuned tiles: their own applies give the batch's results
    for p in plans:
        if p.n_x and p.n_y:
            assert p.tiles() == info["tiles"]
    for i, (a, r) in enumerate(zip(got, _standalone(plans, wus))):
        assert np.array_equal(a, r), i
    # a second batch over the same shapes takes the cached choice without timing
    b2 = ffm.Batch(plans, graph=True, autotune=True, cache=cache)
    i2 = b2.info()
    assert i2["tuned"] == 2 and i2["tiles"] == info["tiles"]
    b2.destroy()


def test_batch_ownership_rules():
    import paper_1909_05600_amd as ffm
    plans, wus, _ = _mixed_instances()
    b = ffm.Batch(plans[:3], graph=False)
    with pytest.raises(ffm.FFMError) as e:
        plans[0].destroy()
    assert e.value.code == -4
    with pytest.raises(ffm.FFMError) as e:
        plans[1].set_tiles(2, 1)
    assert e.value.code == -4
    with pytest.raises(ffm.FFMError) as e:
        ffm.Batch(plans[2:4])
    assert e.value.code == -4
    with pytest.raises(ffm.FFMError) as e:
        ffm.Batch([plans[5], plans[5]])
    assert e.value.code == -1
    b.destroy()
    for p in plans:
        p.destroy()


def test_cfg4_batch_256_instances(orc):
    """The batched workload at full size: 256 instances, N log-uniform in [2e3, 2e5], half Laplace and half
    Helmholtz (k log-uniform in [1, 50]), sphere / ellipsoid / cube.  Graph replay equals every instance's
    own apply bitwise; every instance is within eps of FP64 dense rows on 64 sampled targets."""
    import torch
    import paper_1909_05600_amd as ffm
    ws = W.batched_instances(256, seed=4)
    plans, wus = [], []
    for w in ws:
        plans.append(gpu_plan(w.X, w.X, w.kernel, w.k, w.eps))
        wus.append(torch.from_numpy(w.wu).cuda())
    ref = _standalone(plans, wus)
    b = ffm.Batch(plans, graph=True)
    print("cfg4 batch:", {k: v for k, v in b.info().items() if k != "tuned_ms"})
    outs = b.apply(wus)
    torch.cuda.synchronize()
    worst = 0.0
    for i, (w, o, r) in enumerate(zip(ws, outs, ref)):
        v = o.cpu().numpy()
        assert np.array_equal(v, r), i
        rows = w.rows[:64]
        d = orc.dense_rows(w.X, w.X, w.wu, w.kernel, w.k, rows)
        e = rel(v[rows].astype(np.complex128), d)
        worst = max(worst, e)
        assert e <= w.eps, (i, w.meta, w.n, w.k, e)
    print("cfg4: worst relative error vs dense over 256 instances %.3e" % worst)
    b.destroy()
    for p in plans:
        p.destroy()


def test_apply_batched_entry_point():
    """ffm_apply_batched: complex64 inputs of a plan set in one pass of merged launches, bitwise equal to each
    plan's own apply; a second call with the same set reuses the kept launches, a call with another set
    replaces them, and destroying a plan of the kept set releases it (then the others still apply alone)."""
    import torch
    import paper_1909_05600_amd as ffm
    plans, wus, _ = _mixed_instances()
    wus = [w.to(torch.complex64) for w in wus]
    ref = _standalone(plans, wus)
    for rep in range(2):
        outs = ffm.apply_batched(plans, wus)
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, ref)):
            assert np.array_equal(o.cpu().numpy(), r), (rep, i)
    sub = plans[:4]
    outs = ffm.apply_batched(sub, wus[:4])
    torch.cuda.synchronize()
    for i in range(4):
        assert np.array_equal(outs[i].cpu().numpy(), ref[i]), i
    with pytest.raises(ffm.FFMError) as e:
        ffm.apply_batched([plans[0], plans[0]], [wus[0], wus[0]])      # a plan twice
    assert e.value.code == -1
    plans[0].destroy()                       # held by the kept launches: released first
    assert np.array_equal(_standalone(plans[1:4], wus[1:4])[2], ref[3])
    b = ffm.Batch(plans[1:3], graph=True)    # an explicit batch of plans the kept launches no longer hold
    with pytest.raises(ffm.FFMError) as e:
        ffm.apply_batched(plans[1:3], wus[1:3])
    assert e.value.code == -4
    b.destroy()
    for p in plans[1:]:
        p.destroy()
