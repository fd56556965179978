"""Host-side pieces of the benchmark: the FP64 dense rows it computes on the device for its error figures are
pinned against the oracle's dense definition (run here on CPU tensors), and its roofline work models and CPU
estimate fit are checked on small synthetic inputs."""
import numpy as np
import pytest

import ffm_workloads as W


@pytest.mark.parametrize("kernel,k", [(0, 0.0), (1, 17.5)])
def test_dense_rows_match_the_oracle(orc, kernel, k):
    import torch
    import bench
    w = W.helmholtz_sphere(3000, seed=4, k=k, n_rows=64)
    X = torch.from_numpy(w.X)
    wu = torch.from_numpy(w.wu)
    got = bench.dense_rows_device(X, wu, kernel, k, w.rows, chunk=1000)
    ref = orc.dense_rows(w.X, w.X, w.wu, kernel, k, w.rows)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_launch_work_models():
    import bench
    st = {"order": [0, 0, 10], "nq": [0, 0, 220], "grid_nodes": [0, 0, 32], "grid_width": [0, 0, 5],
          "fwd_boxes": [0, 0, 7], "bwd_boxes": [0, 0, 9], "fwd_points": [0, 0, 1000.0], "bwd_points": [0, 0, 900.0],
          "method": [0, 0, 2], "near_pairs": 5e6, "nclass": [0, 0, 316], "nfar": [0, 0, 100], "_helm": True}
    assert bench.launch_work("k_near<true, false>", 0, st)[0] == 24 * 5e6
    assert bench.launch_work("k_near<false, false>", 0, st)[0] == 14 * 5e6
    assert bench.launch_work("k_near<true, true>", 0, st)[0] == 24 * 5e6
    assert bench.launch_work("k_near_dn<true, false>", 0, st)[0] == 35 * 5e6
    assert bench.launch_work("k_near_dn<false, false>", 0, st)[0] == 21 * 5e6
    assert bench.launch_work("k_near_dl<true, true>", 0, st)[0] == 35 * 5e6
    assert bench.launch_work("k_near_dl<false, false>", 0, st)[0] == 21 * 5e6
    assert bench.launch_work("k_pw_forward_dl<1, 256, false>", 2, st)[0] == 12 * 1000 * 220
    assert bench.launch_work("k_pw_forward<1, 256, false>", 2, st)[0] == 8 * 1000 * 220
    assert bench.launch_work("k_pw_forward_rings<2, false>", 2, st)[0] == 5.5 * 1000 * 220
    assert bench.launch_work("k_pw_backward<256, false>", 2, st)[0] == 8 * 900 * 220
    assert bench.launch_work("k_grid_phit", 2, st)[0] == 8 * 9 * 11 * 32 * 32 * 10
    assert bench.launch_work("k_grid_z", 2, st)[0] == 8 * 7 * 6 * 32 ** 3
    assert bench.launch_work("k_sum_segments", 2, st) is None
