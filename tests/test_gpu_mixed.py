"""Mixed precision: Lagrange transfers on FP16 MFMA with FP32 accumulation (ffm_options_t.precision =
FFM_PREC_MIXED), chosen per level at plan time; Gegenbauer levels stay FP32.

Errors are stated against the FP64 oracle: relative L2 vs FP64 dense rows <= eps, and vs the oracle FFM
within the FP16 rounding budget (2^-11 times the kernel's conditioning factor).
Paper: Sec. 2.2.2 (Lagrange transfer T), Sec. 4.1 (workloads); the paper ran single precision throughout.
"""
import numpy as np
import pytest

import ffm_workloads as W
from gpu_common import FP32_RTOL, gpu_apply, gpu_plan, oracle_like, rel

pytestmark = pytest.mark.gpu
MIXED = 1


@pytest.mark.parametrize("eps", [1e-3, 1e-4])
def test_mixed_laplace(orc, eps):
    w = W.laplace_sphere(20000, seed=17, eps=eps)
    gp = gpu_plan(w.X, w.X, 0, 0.0, eps, precision=MIXED)
    st = gp.stats()
    lag = [l for l in range(1, st["leaf"] + 1) if st["method"][l] == 1]
    assert lag
    expect_fp16 = eps >= 2.0 ** -11
    assert all(st["prec"][l] == (1 if expect_fp16 else 0) for l in lag), st["prec"]
    v = gpu_apply(gp, w.wu)
    vo = oracle_like(orc, gp, w.X, w.X, 0, 0.0, eps).apply(w.wu)
    d = orc.dense_rows(w.X, w.X, w.wu, 0, 0.0, w.rows[:2048])
    e_o, e_d = rel(v, vo), rel(v[w.rows[:2048]], d)
    print("mixed laplace eps=%g fp16=%s: vs oracle %.3e vs dense %.3e" % (eps, expect_fp16, e_o, e_d))
    assert e_d <= eps
    assert e_o <= (2.0 ** -11 if expect_fp16 else FP32_RTOL)
    if not expect_fp16:
        # no FP16 level: the mixed plan runs exactly the FP32 kernels
        assert np.array_equal(v, gpu_apply(gpu_plan(w.X, w.X, 0, 0.0, eps), w.wu))


def test_mixed_helmholtz_low_frequency(orc):
    rng = np.random.default_rng(12)
    X = W.sphere_points(20000, rng)
    wu = ((rng.standard_normal(20000) + 1j * rng.standard_normal(20000)) / 20000).astype(np.complex64)
    gp = gpu_plan(X, X, 1, 9.0, 1e-3, precision=MIXED)
    st = gp.stats()
    assert any(st["prec"][l] == 1 for l in range(1, st["leaf"] + 1))
    assert all(st["prec"][l] == 0 for l in range(1, st["leaf"] + 1) if st["method"][l] == 2)
    v = gpu_apply(gp, wu)
    vo = oracle_like(orc, gp, X, X, 1, 9.0, 1e-3).apply(wu)
    rows = np.arange(0, 20000, 13)
    d = orc.dense_rows(X, X, wu, 1, 9.0, rows)
    print("mixed helmholtz k=9: vs oracle %.3e vs dense %.3e" % (rel(v, vo), rel(v[rows], d)))
    assert rel(v[rows], d) <= 1e-3
    assert rel(v, vo) <= 2 * 2.0 ** -11


def test_mixed_is_deterministic_and_matches_fp32_structure(orc):
    w = W.laplace_sphere(30000, seed=3)
    a = gpu_plan(w.X, w.X, 0, 0.0, 1e-3, precision=MIXED)
    b = gpu_plan(w.X, w.X, 0, 0.0, 1e-3)
    sa, sb = a.stats(), b.stats()
    assert sa["nfar"] == sb["nfar"] and sa["leaf"] == sb["leaf"]
    v1, v2 = gpu_apply(a, w.wu), gpu_apply(a, w.wu)
    assert np.array_equal(v1, v2)
    vf = gpu_apply(b, w.wu)
    assert rel(v1, vf) <= 2.0 ** -11


@pytest.mark.parametrize("eps", [1e-3, 1e-4])
@pytest.mark.parametrize("precision", [0, MIXED])
def test_sphere_plus_cube_cluster(orc, eps, precision):
    """The non-uniform workload (80% on the sphere, 20% in a cube cluster) at 1/10 of its size: errors vs
    FP64 dense rows overall and per target class, for both precision modes."""
    w = W.sphere_plus_cube(1_000_000, seed=3, eps=eps, n_rows=512)
    gp = gpu_plan(w.X, w.X, 1, w.k, eps, precision=precision)
    v = gpu_apply(gp, w.wu)
    d = orc.dense_rows(w.X, w.X, w.wu, 1, w.k, w.rows)
    sph = w.rows < w.meta["n_sphere"]
    e_all, e_s, e_c = rel(v[w.rows], d), rel(v[w.rows][sph], d[sph]), rel(v[w.rows][~sph], d[~sph])
    print("sphere+cube N=%d eps=%g prec=%d: all %.3e sphere %.3e cube %.3e" % (w.n, eps, precision, e_all, e_s, e_c))
    assert e_all <= eps and e_s <= eps and e_c <= eps
