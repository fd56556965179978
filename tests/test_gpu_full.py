"""Full-size parity at the benchmark workload (N = 1,048,576 Helmholtz on the unit sphere, k for ten
points per wavelength, eps = 1e-3), in the launch configuration bench.py times (default options).

Outputs the oracle computes one by one: FP64 dense rows on 4096 sampled targets (relative L2 <= eps).
Bit-exact: Morton keys, permutation, boxes and descent lists of every level against the oracle plan.
Paper: Sec. 4.1 (Table validationHelmholtz reports 2.8e-4 at N = 1e6, k r_max = 200, eps = 1e-3).
"""
import numpy as np
import pytest

import ffm_workloads as W
from gpu_common import compare_trees, gpu_apply, gpu_plan, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cfg2():
    return W.helmholtz_sphere(1 << 20, seed=2)


def test_helmholtz_1M_tree_bit_exact(orc, cfg2):
    w = cfg2
    gp = gpu_plan(w.X, w.X, 1, w.k, w.eps)
    op = orc.Plan(w.X, w.X, 1, w.k, w.eps)
    st = gp.stats()
    print("leaf %d, nbox %s, nfar %s, nq %s" % (st["leaf"], st["nbox_x"][:st["leaf"] + 1],
                                                st["nfar"][:st["leaf"] + 1], st["nq"][:st["leaf"] + 1]))
    compare_trees(gp, op)


def test_helmholtz_1M_error_vs_dense(orc, cfg2):
    w = cfg2
    gp = gpu_plan(w.X, w.X, 1, w.k, w.eps)
    v = gpu_apply(gp, w.wu)
    d = orc.dense_rows(w.X, w.X, w.wu, 1, w.k, w.rows)
    e = rel(v[w.rows], d)
    print("N=%d k=%.3f: relative L2 error on %d rows vs FP64 dense = %.3e" % (w.n, w.k, len(w.rows), e))
    assert e <= w.eps
    # a second apply on the same plan is bitwise identical (owner-computes, fixed summation order)
    v2 = gpu_apply(gp, w.wu)
    assert np.array_equal(v, v2)
