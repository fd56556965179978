"""The per-pair leaf rule on the GPU (beyond the global stopping rule of Sec. 2.2.4): near pairs whose two
boxes both hold at most n_leaf points are summed densely at their level.  On the non-uniform cloud of the
mixed-precision workload (80% on the sphere, 20% in a cube cluster) at reduced size: the lists of every
level, the early lists included, bit-exact against the oracle; the product element-wise against the oracle
with identical parameters (FP32_RTOL) and within eps of FP64 dense rows per target class."""
import numpy as np
import pytest

import ffm_workloads as W
from gpu_common import FP32_RTOL, compare_trees, gpu_apply, gpu_plan, oracle_like, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,eps,kernel", [(100000, 1e-3, 1), (60000, 1e-4, 1), (60000, 1e-3, 0)])
def test_adaptive_leaves_match_oracle(orc, n, eps, kernel):
    import paper_1909_05600_amd as ffm
    w = W.sphere_plus_cube(n, seed=3, eps=eps, n_rows=384)
    k = w.k if kernel == 1 else 0.0
    gp = gpu_plan(w.X, w.X, kernel, k, eps, adaptive=True)
    st = gp.stats()
    op = oracle_like(orc, gp, w.X, w.X, kernel, k, eps, adaptive=True)
    compare_trees(gp, op)
    for l in range(1, st["leaf"] + 1):
        g = gp.export(ffm.FFM_EXPORT_EARLY, 0, l)
        t, s = op.early(l)
        assert np.array_equal(g[:, 0], t) and np.array_equal(g[:, 1], s), l
    assert sum(st["nearly"]) > 0, st["nearly"]
    v = gpu_apply(gp, w.wu)
    vo = op.apply(w.wu)
    d = orc.dense_rows(w.X, w.X, w.wu, kernel, k, w.rows)
    vp = gpu_apply(gpu_plan(w.X, w.X, kernel, k, eps), w.wu)
    sph = w.rows < w.meta["n_sphere"]
    e_all, e_s, e_c = rel(v[w.rows], d), rel(v[w.rows][sph], d[sph]), rel(v[w.rows][~sph], d[~sph])
    print("adaptive N=%d kernel %d eps=%g: early pairs per level %s, leaf %d: vs oracle %.3e, vs dense %.3e "
          "(sphere %.3e, cube %.3e), vs plain descent %.3e"
          % (n, kernel, eps, st["nearly"][:st["leaf"] + 1], st["leaf"], rel(v, vo), e_all, e_s, e_c, rel(v, vp)))
    assert rel(v, vo) < FP32_RTOL
    assert e_all <= eps and e_s <= eps and e_c <= eps
    assert np.array_equal(v, gpu_apply(gp, w.wu))
