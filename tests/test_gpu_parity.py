"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

Tree, Morton keys, permutation, boxes and descent lists: bit-exact.
v: element-wise against the oracle FFM with identical parameters (relative L2 within FP32_RTOL = 1e-5, the
grid form's levels included: the oracle then runs the same grid) and against FP64 dense rows (relative
L2 <= eps).
Paper: Sec. 2.2 (algorithm), Sec. 4.1 (workloads: random points on the unit sphere, eps = 1e-3).
"""
import math

import numpy as np
import pytest

import ffm_workloads as W
from gpu_common import FP32_RTOL, compare_trees, gpu_apply, gpu_plan, oracle_like, rel

pytestmark = pytest.mark.gpu


def _shifted_sets(n, m, seed):
    rng = np.random.default_rng(seed)
    X = W.sphere_points(n, rng)
    Y = W.sphere_points(m, rng) * 0.97 + np.array([0.01, -0.02, 0.005])
    wu = ((rng.standard_normal(m) + 1j * rng.standard_normal(m)) / m).astype(np.complex64)
    return X, Y, wu


def test_laplace_sphere_4096(orc):
    """N = 4096 Laplace, same set, real FP64 u: the correctness workload."""
    w = W.laplace_sphere(4096, seed=1)
    gp = gpu_plan(w.X, w.X, 0, 0.0, w.eps)
    op = oracle_like(orc, gp, w.X, w.X, 0, 0.0, w.eps)
    compare_trees(gp, op)
    v = gpu_apply(gp, w.wu)
    vo = op.apply(w.wu)
    d = orc.dense_rows(w.X, w.X, w.wu, 0, 0.0, np.arange(w.n))
    print("laplace 4096: vs oracle %.3e  vs dense %.3e (oracle %.3e)" % (rel(v, vo), rel(v, d), rel(vo, d)))
    assert rel(v, vo) < FP32_RTOL
    assert rel(v, d) <= w.eps


@pytest.mark.parametrize("n,seed", [(4096, 2), (16384, 3), (40000, 4)])
def test_helmholtz_sphere(orc, n, seed):
    w = W.helmholtz_sphere(n, seed=seed, n_rows=512)
    gp = gpu_plan(w.X, w.X, 1, w.k, w.eps)
    op = oracle_like(orc, gp, w.X, w.X, 1, w.k, w.eps)
    compare_trees(gp, op)
    v = gpu_apply(gp, w.wu)
    vo = op.apply(w.wu)
    d = orc.dense_rows(w.X, w.X, w.wu, 1, w.k, w.rows)
    print("helmholtz %d k=%.2f: vs oracle %.3e  vs dense %.3e (oracle %.3e)"
          % (n, w.k, rel(v, vo), rel(v[w.rows], d), rel(vo[w.rows], d)))
    assert rel(v, vo) < FP32_RTOL
    assert rel(v[w.rows], d) <= w.eps


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 5.0), (1, 40.0)])
def test_shifted_trees(orc, kernel, k):
    """Different source and target sets: root cubes are translates; FP64 far test; classes off-centre."""
    X, Y, wu = _shifted_sets(6000, 5000, 31)
    gp = gpu_plan(X, Y, kernel, k, 1e-3, n_leaf=32)
    op = oracle_like(orc, gp, X, Y, kernel, k, 1e-3, n_leaf=32)
    compare_trees(gp, op)
    v = gpu_apply(gp, wu)
    vo = op.apply(wu)
    d = orc.dense_rows(X, Y, wu, kernel, k, np.arange(0, 6000, 7))
    print("shifted k=%.1f: vs oracle %.3e vs dense %.3e" % (k, rel(v, vo), rel(v[::7], d)))
    assert rel(v, vo) < FP32_RTOL
    assert rel(v[::7], d) <= 1e-3


def test_helmholtz_lagrange_levels(orc):
    """Low frequency: Helmholtz levels with k d_l < pi use complex Lagrange transfers (MFMA)."""
    rng = np.random.default_rng(12)
    X = W.sphere_points(20000, rng)
    wu = ((rng.standard_normal(20000) + 1j * rng.standard_normal(20000)) / 20000).astype(np.complex64)
    gp = gpu_plan(X, X, 1, 9.0, 1e-3)
    op = oracle_like(orc, gp, X, X, 1, 9.0, 1e-3)
    st = gp.stats()
    assert 1 in st["method"] and 2 in st["method"], st["method"]
    compare_trees(gp, op)
    v = gpu_apply(gp, wu)
    vo = op.apply(wu)
    assert rel(v, vo) < FP32_RTOL


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-5])
def test_laplace_other_eps(orc, eps):
    w = W.laplace_sphere(8192, seed=7, eps=eps)
    gp = gpu_plan(w.X, w.X, 0, 0.0, eps)
    op = oracle_like(orc, gp, w.X, w.X, 0, 0.0, eps)
    v = gpu_apply(gp, w.wu)
    vo = op.apply(w.wu)
    d = orc.dense_rows(w.X, w.X, w.wu, 0, 0.0, w.rows[:1024])
    print("laplace eps=%g: vs oracle %.3e vs dense %.3e" % (eps, rel(v, vo), rel(v[w.rows[:1024]], d)))
    assert rel(v, vo) < FP32_RTOL
    assert rel(v[w.rows[:1024]], d) <= max(eps, 3e-6)


def test_near_field_only_equals_dense(orc):
    """A plan with no admissible pair (n_leaf >= N) is the dense sum: only the near-field kernel runs."""
    for kernel, k in ((0, 0.0), (1, 7.5)):
        w = W.helmholtz_sphere(3000, seed=9, k=k)
        gp = gpu_plan(w.X, w.X, kernel, k, 1e-3, n_leaf=10 ** 6)
        assert gp.stats()["leaf"] == 1 and sum(gp.stats()["nfar"]) == 0
        v = gpu_apply(gp, w.wu)
        d = orc.dense_rows(w.X, w.X, w.wu, kernel, k, np.arange(w.n))
        # FP32 accumulation of ~3000 terms: relative error ~ sqrt(n) * 2^-24 = 3.3e-6
        assert rel(v, d) < 1e-5, rel(v, d)


def test_apply_is_deterministic(orc):
    w = W.helmholtz_sphere(30000, seed=5)
    gp = gpu_plan(w.X, w.X, 1, w.k, w.eps)
    a = gpu_apply(gp, w.wu)
    b = gpu_apply(gp, w.wu)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.complex64, np.complex128])
def test_input_dtypes(orc, dtype):
    rng = np.random.default_rng(3)
    X = W.sphere_points(2000, rng)
    u = rng.standard_normal(2000) + (1j * rng.standard_normal(2000) if np.iscomplexobj(dtype(0)) else 0)
    wu = (u / 2000).astype(dtype)
    gp = gpu_plan(X, X, 1, 6.0, 1e-3)
    v = gpu_apply(gp, wu)
    vo = oracle_like(orc, gp, X, X, 1, 6.0, 1e-3).apply(wu.astype(np.complex128))
    assert rel(v, vo) < FP32_RTOL


def test_edge_cases(orc):
    import torch
    import paper_1909_05600_amd as ffm
    # a single point: no interaction at all
    P = np.array([[0.1, 0.2, 0.3]])
    gp = gpu_plan(P, P, 1, 3.0, 1e-3)
    assert np.all(gpu_apply(gp, np.array([1.0 + 1j], dtype=np.complex64)) == 0)
    # empty source set: v = 0; empty target set: nothing to write
    X = W.sphere_points(100, np.random.default_rng(1))
    E = np.zeros((0, 3))
    gp = gpu_plan(X, E, 0, 0.0, 1e-3)
    v = gp.apply(torch.zeros(0, dtype=torch.complex64, device="cuda"))
    assert torch.count_nonzero(v).item() == 0 and v.shape[0] == 100
    # duplicated points are coincident: excluded, like the self term
    rng = np.random.default_rng(2)
    Q = W.sphere_points(3000, rng)
    Q = np.concatenate([Q, Q[:500]])
    wu = (rng.standard_normal(3500) / 3500).astype(np.float64)
    gp = gpu_plan(Q, Q, 1, 12.0, 1e-3, n_leaf=16)
    op = oracle_like(orc, gp, Q, Q, 1, 12.0, 1e-3, n_leaf=16)
    compare_trees(gp, op)
    assert rel(gpu_apply(gp, wu), op.apply(wu)) < FP32_RTOL
    # NaN coordinates are rejected
    Bad = X.copy()
    Bad[7, 1] = np.nan
    with pytest.raises(ffm.FFMError):
        gpu_plan(Bad, Bad, 0, 0.0, 1e-3)


def test_ragged_and_unequal_sizes(orc):
    """Targets and sources of different sizes, a cube cluster (non-uniform tree), ragged leaves."""
    rng = np.random.default_rng(77)
    X = np.concatenate([W.sphere_points(7001, rng), W.cube_points(1999, rng, (0.3, -0.2, 0.1), 0.4)])
    Y = np.concatenate([W.sphere_points(5003, rng), W.cube_points(3001, rng, (0.3, -0.2, 0.1), 0.4)])
    wu = ((rng.standard_normal(8004) + 1j * rng.standard_normal(8004)) / 8004).astype(np.complex64)
    for kernel, k in ((0, 0.0), (1, 20.0)):
        gp = gpu_plan(X, Y, kernel, k, 1e-3, n_leaf=40)
        op = oracle_like(orc, gp, X, Y, kernel, k, 1e-3, n_leaf=40)
        compare_trees(gp, op)
        assert rel(gpu_apply(gp, wu), op.apply(wu)) < FP32_RTOL


@pytest.mark.parametrize("eps", [1e-3, 1e-4])
def test_ring_pair_transforms(orc, eps):
    """Coarse Gegenbauer levels with long rings use the ring-pair transform kernels (4 directions per
    sin/cos); at eps = 1e-4 the in-plane phase is reduced in FP64, at 1e-3 in FP32."""
    rng = np.random.default_rng(21)
    X = W.sphere_points(50000, rng)
    wu = ((rng.standard_normal(50000) + 1j * rng.standard_normal(50000)) / 50000).astype(np.complex64)
    k = 100.0
    gp = gpu_plan(X, X, 1, k, eps, transforms="direct")
    op = oracle_like(orc, gp, X, X, 1, k, eps)
    st = gp.stats()
    assert max(st["order"]) >= 64 and 2 in st["tform"], st["tform"]
    compare_trees(gp, op)
    v = gpu_apply(gp, wu)
    vo = op.apply(wu)
    rows = np.arange(0, 50000, 97)
    d = orc.dense_rows(X, X, wu, 1, k, rows)
    print("ring-pair eps=%g: vs oracle %.3e  vs dense %.3e (oracle %.3e)"
          % (eps, rel(v, vo), rel(v[rows], d), rel(vo[rows], d)))
    assert rel(v, vo) < FP32_RTOL
    assert rel(v[rows], d) <= eps


def test_plan_tail_runs_ahead_of_the_caller():
    """ffm_plan returns with its last tables and launch lists still running on the planning stream.  An apply
    on another stream issued at once (ordered by the plan's readiness event on the device), an export, a
    second plan and a destroy right after planning all see a complete plan: results equal those of a plan
    whose stream was synchronised first, bitwise."""
    import torch
    import paper_1909_05600_amd as ffm
    w = W.helmholtz_sphere(200000, seed=12, k=80.0)
    X = torch.from_numpy(w.X).cuda()
    wu = torch.from_numpy(w.wu).cuda()
    s_plan, s_apply = torch.cuda.Stream(), torch.cuda.Stream()
    ref_plan = ffm.Plan(X, X, 1, w.k, w.eps, stream=s_plan)
    torch.cuda.synchronize()
    ref = ref_plan.apply(wu)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    keys_ref = ref_plan.export(ffm.FFM_EXPORT_FAR, 0, ref_plan.stats()["leaf"])
    for rep in range(3):
        p = ffm.Plan(X, X, 1, w.k, w.eps, stream=s_plan)
        with torch.cuda.stream(s_apply):
            out = torch.empty(w.n, dtype=torch.complex64, device="cuda")
        v = p.apply(wu, out=out, stream=s_apply)          # no host synchronisation in between
        s_apply.synchronize()
        assert np.array_equal(v.cpu().numpy(), ref), rep
        q = ffm.Plan(X, X, 1, w.k, w.eps, stream=s_plan)   # export before any apply
        assert np.array_equal(q.export(ffm.FFM_EXPORT_FAR, 0, q.stats()["leaf"]), keys_ref)
        q.destroy()
        ffm.Plan(X, X, 1, w.k, w.eps, stream=s_plan).destroy()   # destroy with the tail still running
        p.destroy()
    ref_plan.destroy()


@pytest.mark.parametrize("transforms", ["direct", "grid"])
def test_headline_wavenumber_levels(orc, transforms):
    """The headline wavenumber k = 2 pi sqrt(2^20 / 4 pi) / 10 = 181.499 on 32,768 sphere points: the tree stops
    at level 4 and levels 2-4 are the headline's Gegenbauer levels (L = 164, 85, 46; the same ring-pair kernels,
    grids and FP64-phase decisions as at N = 2^20).  Both transform forms, element-wise against the oracle FFM
    with identical parameters, and within eps of FP64 dense rows."""
    k = 2.0 * math.pi * math.sqrt((1 << 20) / (4.0 * math.pi)) / 10.0
    w = W.helmholtz_sphere(32768, seed=2, k=k, n_rows=384)
    gp = gpu_plan(w.X, w.X, 1, w.k, w.eps, transforms=transforms)
    st = gp.stats()
    assert st["leaf"] == 4 and st["order"][2:5] == [164, 85, 46], (st["leaf"], st["order"])
    if transforms == "grid":
        assert st["tform"][2:5] == [3, 3, 3], st["tform"]
    else:
        assert all(t in (1, 2) for t in st["tform"][2:5]), st["tform"]
    op = oracle_like(orc, gp, w.X, w.X, 1, w.k, w.eps)
    compare_trees(gp, op)
    v = gpu_apply(gp, w.wu)
    vo = op.apply(w.wu)
    d = orc.dense_rows(w.X, w.X, w.wu, 1, w.k, w.rows)
    print("headline k, %s transforms (forms %s, grids %s, FP64 phases %s): vs oracle %.3e  vs dense %.3e (oracle %.3e)"
          % (transforms, st["tform"][2:5], st["grid_nodes"][2:5], st["phase64"][2:5], rel(v, vo), rel(v[w.rows], d),
             rel(vo[w.rows], d)))
    assert rel(v, vo) < FP32_RTOL
    assert rel(v[w.rows], d) <= w.eps


def test_shifted_quadtree_lists_bit_exact(orc):
    """Points on a plane with the source tree shifted by half a box of level 4 (the shifted configuration of the
    proof of Prop. 1, Sec. 3.2): the GPU's lists equal the oracle's bitwise, and an interior target box has 48 far
    interactions."""
    rng = np.random.default_rng(5)
    m = 16

    def grid(seed):
        r = np.random.default_rng(seed)
        idx = np.stack(np.meshgrid(np.arange(m), np.arange(m), indexing="ij"), axis=-1).reshape(-1, 2)
        P = (idx + 0.1 + 0.8 * r.random(idx.shape)) / m
        P = np.concatenate([P, [[0.0, 0.0], [0.0, 1.0], [1.0, 0.0], [1.0, 1.0]]])
        return np.concatenate([P, np.zeros((P.shape[0], 1))], axis=1)

    X, Y = grid(5), grid(6) + np.array([0.5 / m, 0.5 / m, 0.0])
    gp = gpu_plan(X, Y, 0, 0.0, 1e-3, n_leaf=1, max_level=5)
    op = orc.Plan(X, Y, 0, 0.0, 1e-3, n_leaf=1, max_level=5)
    compare_trees(gp, op)
    import paper_1909_05600_amd as ffm
    far = gp.export(ffm.FFM_EXPORT_FAR, 0, 4)
    ijk = gp.export(ffm.FFM_EXPORT_BOX_IJK, 0, 4)
    counts = np.bincount(far[:, 0], minlength=ijk.shape[0])
    interior = np.all((ijk[:, :2] >= 5) & (ijk[:, :2] <= 10), axis=1)
    assert np.all(counts[interior] == 48) and counts.max() == 48
    wu = ((rng.standard_normal(Y.shape[0]) + 1j * rng.standard_normal(Y.shape[0])) / Y.shape[0]).astype(np.complex64)
    assert rel(gpu_apply(gp, wu), op.apply(wu)) < FP32_RTOL
