"""Grid form of the plane-wave transforms: source points spread onto a uniform grid with a smooth kernel,
separable sums from the grid to the quadrature directions, the kernel's Fourier transform divided out in
the transfer; the mirror steps at the targets (the fast evaluation of the transforms that the remark
closing Sec. 2.2.3 calls for).  Parity with the FP64 oracle FFM running the same grids (same p, w, beta: FP32
rounding alone separates the two, bound FP32_RTOL) and with its direct transforms (within the aliasing bound
2 E, E = (1 + B)^3 - 1 from the plan's own per-level bound B), FP64 dense rows, agreement with the direct GPU
transforms, bitwise determinism, and the planner's choice at full size."""
import numpy as np
import pytest

import ffm_workloads as W
from gpu_common import FP32_RTOL, compare_trees, gpu_apply, gpu_plan, oracle_grid, oracle_like, rel


pytestmark = pytest.mark.gpu


def alias_bound(gp) -> float:
    """2 E: one grid transform on each side of the transfer, E = (1 + B)^3 - 1 per transform (three axes)."""
    B = max(gp.stats()["grid_alias"])
    return 2.0 * ((1.0 + B) ** 3 - 1.0)


@pytest.mark.parametrize("n,k,seed,eps", [(40000, 100.0, 7, 1e-3), (30000, 45.0, 8, 1e-3), (30000, 60.0, 9, 1e-4)])
def test_grid_matches_oracle_and_dense(orc, n, k, seed, eps):
    w = W.helmholtz_sphere(n, seed=seed, k=k, eps=eps, n_rows=512)
    gp = gpu_plan(w.X, w.X, 1, w.k, w.eps, transforms="grid")
    st = gp.stats()
    grid_levels = [l for l in range(1, st["leaf"] + 1) if st["tform"][l] == 3]
    assert grid_levels, st["tform"]
    op = oracle_like(orc, gp, w.X, w.X, 1, w.k, w.eps)
    compare_trees(gp, op, levels=[st["leaf"]])
    v = gpu_apply(gp, w.wu)
    vo = op.apply(w.wu)
    vod = orc.Plan(w.X, w.X, 1, w.k, w.eps).apply(w.wu)      # the oracle's direct transforms
    d = orc.dense_rows(w.X, w.X, w.wu, 1, w.k, w.rows)
    vd = gpu_apply(gpu_plan(w.X, w.X, 1, w.k, w.eps, transforms="direct"), w.wu)
    print("grid levels %s %s: vs oracle (same grids) %.3e, vs oracle direct %.3e (bound %.3e), vs dense %.3e, "
          "vs direct GPU %.3e" % (grid_levels, oracle_grid(gp), rel(v, vo), rel(v, vod), alias_bound(gp),
                                   rel(v[w.rows], d), rel(v, vd)))
    assert rel(v, vo) < FP32_RTOL
    assert rel(v, vod) < alias_bound(gp)
    assert rel(v[w.rows], d) <= w.eps
    # both forms are within eps of the product; the grid form keeps its aliasing bound (one axis, worst
    # direction) at eps / 2, and products measure well under a third of that: the two agree to eps / 4
    assert rel(v, vd) < w.eps / 4
    assert np.array_equal(v, gpu_apply(gp, w.wu))


@pytest.mark.parametrize("k", [280.0, 350.0, 415.0, 480.0])
def test_grid_large_grids(orc, k):
    """Level 2 on grids of 80 to 128 nodes per axis (wavenumbers of 280 to 480 on the unit sphere; the plane sums
    hold each wave's grid rows in registers): within eps of FP64 dense rows, within eps / 4 of the direct GPU
    transforms, bitwise repeatable."""
    w = W.helmholtz_sphere(20000, seed=31, k=k, n_rows=512)
    gp = gpu_plan(w.X, w.X, 1, w.k, w.eps, transforms="grid")
    st = gp.stats()
    assert st["tform"][2] == 3 and st["grid_nodes"][2] > 64, (st["tform"], st["grid_nodes"])
    v = gpu_apply(gp, w.wu)
    d = orc.dense_rows(w.X, w.X, w.wu, 1, w.k, w.rows)
    vd = gpu_apply(gpu_plan(w.X, w.X, 1, w.k, w.eps, transforms="direct"), w.wu)
    print("k %.0f: level-2 grid %d nodes (w = %d): vs dense %.3e vs direct GPU %.3e"
          % (k, st["grid_nodes"][2], st["grid_width"][2], rel(v[w.rows], d), rel(v, vd)))
    assert rel(v[w.rows], d) <= w.eps
    assert rel(v, vd) < w.eps / 4
    assert np.array_equal(v, gpu_apply(gp, w.wu))


def test_grid_shifted_trees(orc):
    """Distinct source and target sets (translated root cubes, FP64 far test)."""
    rng = np.random.default_rng(21)
    X = W.sphere_points(9000, rng)
    Y = W.sphere_points(8000, rng) * 0.95 + np.array([0.02, -0.01, 0.03])
    wu = ((rng.standard_normal(8000) + 1j * rng.standard_normal(8000)) / 8000).astype(np.complex64)
    gp = gpu_plan(X, Y, 1, 40.0, 1e-3, transforms="grid")
    assert 3 in gp.stats()["tform"]
    v = gpu_apply(gp, wu)
    vo = oracle_like(orc, gp, X, Y, 1, 40.0, 1e-3).apply(wu)
    rows = np.arange(0, 9000, 23)
    d = orc.dense_rows(X, Y, wu, 1, 40.0, rows)
    print("shifted grid: vs oracle %.3e vs dense %.3e" % (rel(v, vo), rel(v[rows], d)))
    assert rel(v, vo) < FP32_RTOL
    assert rel(v[rows], d) <= 1e-3


def test_grid_zero_and_scaled_input():
    """The fixed-point spreading scales with max |u|: zero input gives zero, and the product is linear."""
    w = W.helmholtz_sphere(20000, seed=5, k=70.0)
    gp = gpu_plan(w.X, w.X, 1, w.k, w.eps, transforms="grid")
    assert 3 in gp.stats()["tform"]
    assert not np.any(gpu_apply(gp, np.zeros_like(w.wu)))
    v1 = gpu_apply(gp, w.wu)
    v2 = gpu_apply(gp, (w.wu * np.float32(2.0 ** -30)).astype(np.complex64))
    assert rel(v2 * 2.0 ** 30, v1) < 1e-6


def test_planner_choice_full_size(orc):
    """N = 1,048,576 Helmholtz: the planner's forms per level; the product within eps of FP64 dense rows and
    within the FP32 tolerance of the all-direct product."""
    w = W.helmholtz_sphere(1 << 20, seed=2, n_rows=1024)
    ga = gpu_plan(w.X, w.X, 1, w.k, w.eps)
    st = ga.stats()
    print("forms per level:", st["tform"][:st["leaf"] + 1])
    va = gpu_apply(ga, w.wu)
    vd = gpu_apply(gpu_plan(w.X, w.X, 1, w.k, w.eps, transforms="direct"), w.wu)
    d = orc.dense_rows(w.X, w.X, w.wu, 1, w.k, w.rows)
    print("auto vs dense %.3e, vs direct %.3e" % (rel(va[w.rows], d), rel(va, vd)))
    assert rel(va[w.rows], d) <= w.eps
    assert rel(va, vd) < w.eps / 4      # as in test_grid_matches_oracle_and_dense
