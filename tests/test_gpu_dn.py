"""The normal derivative at the target, dG/dn_x (x, y) = n_x . grad_x G(x - y): the kernel of the adjoint
double-layer operator (Sec. 4.2.1, eq. doubleLayer), on the GPU through the C ABI (FFM_LAPLACE_DN,
FFM_HELMHOLTZ_DN with target normals).

Only the target side differs from the potential: the near-field kernel, the derivatives of the Lagrange
polynomials at the targets, and the factor ik (s . n) of every plane wave: in direction pairs, or, where the
target transform takes the ring-pair or the grid form, as n . (the plain target transforms of ik s_c v~, c = 0, 1,
2).  Element-wise against the oracle FFM of the same kernel with identical parameters, grid-form levels included
(FP32_RTOL), within eps of FP64 dense rows, bitwise repeatable, inside a batch, and the missing-normals error.
"""
import numpy as np
import pytest

import ffm_workloads as W
from gpu_common import FP32_RTOL, compare_trees, gpu_apply, oracle_like, rel

pytestmark = pytest.mark.gpu


def _plan(X, Y, kernel, k, eps, N, **kw):
    import torch
    import paper_1909_05600_amd as ffm
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Yd = Xd if Y is X else torch.from_numpy(np.ascontiguousarray(Y)).cuda()
    Nd = torch.from_numpy(np.ascontiguousarray(N)).cuda()
    return ffm.Plan(Xd, Yd, kernel, k, eps, normals=Nd, **kw)


@pytest.mark.parametrize("kernel,k,eps,tf", [(2, 0.0, 1e-3, "auto"), (2, 0.0, 1e-4, "auto"), (3, 9.0, 1e-3, "auto"),
                                             (3, 45.0, 1e-3, "auto"), (3, 20.0, 1e-4, "auto"), (3, 45.0, 1e-3, "grid"),
                                             (3, 60.0, 1e-4, "grid")])
def test_dn_matches_oracle_and_dense(orc, kernel, k, eps, tf):
    rng = np.random.default_rng(int(k) + 7)
    Y = W.sphere_points(20000, rng)
    N = W.sphere_points(15000, rng)
    X = N * 0.985                                     # targets just inside the sources' sphere, radial normals
    wu = ((rng.standard_normal(20000) + 1j * rng.standard_normal(20000)) / 20000).astype(np.complex64)
    print("dn kernel %d k=%g eps=%g transforms %s" % (kernel, k, eps, tf), flush=True)
    gp = _plan(X, Y, kernel, k, eps, N, transforms=tf)
    st = gp.stats()
    op = oracle_like(orc, gp, X, Y, kernel, k, eps, normals=N)
    compare_trees(gp, op)
    v = gpu_apply(gp, wu)
    vo = op.apply(wu)
    rows = np.arange(0, 15000, 29)
    d = orc.dense_rows_dn(X, Y, wu, kernel - 2, k, N, rows)
    print("dn kernel %d k=%g eps=%g: methods %s forms %s aca %s: vs oracle %.3e, vs dense %.3e (oracle %.3e)"
          % (kernel, k, eps, st["method"][:st["leaf"] + 1], st["tform"][:st["leaf"] + 1], st["aca"][:st["leaf"] + 1],
             rel(v, vo), rel(v[rows], d), rel(vo[rows], d)))
    if tf == "grid":
        assert 3 in st["tform"], st["tform"]
    assert rel(v, vo) < FP32_RTOL
    assert rel(v[rows], d) <= eps
    assert np.array_equal(v, gpu_apply(gp, wu))


def test_dn_same_set_and_batch(orc):
    """One set with its own normals (the self term excluded), and a batch mixing a normal-derivative plan with
    a potential plan: each instance bitwise its own apply."""
    import torch
    import paper_1909_05600_amd as ffm
    rng = np.random.default_rng(3)
    X = W.sphere_points(12000, rng)
    wu = ((rng.standard_normal(12000) + 1j * rng.standard_normal(12000)) / 12000).astype(np.complex64)
    Xd = torch.from_numpy(X).cuda()
    gp = ffm.Plan(Xd, Xd, 3, 15.0, 1e-3, normals=Xd)
    v = gpu_apply(gp, wu)
    vo = oracle_like(orc, gp, X, X, 3, 15.0, 1e-3, normals=X).apply(wu)
    assert rel(v, vo) < FP32_RTOL
    other = ffm.Plan(Xd, Xd, 1, 15.0, 1e-3)
    ref_other = gpu_apply(other, wu)
    w = torch.from_numpy(wu).cuda()
    b = ffm.Batch([gp, other], graph=True)
    outs = b.apply([w, w])
    torch.cuda.synchronize()
    assert np.array_equal(outs[0].cpu().numpy().astype(np.complex128), v)
    assert np.array_equal(outs[1].cpu().numpy().astype(np.complex128), ref_other)
    b.destroy()


def test_dn_needs_normals():
    import torch
    import paper_1909_05600_amd as ffm
    X = torch.from_numpy(W.sphere_points(500, np.random.default_rng(1))).cuda()
    with pytest.raises(ffm.FFMError) as e:
        ffm.Plan(X, X, ffm.FFM_HELMHOLTZ_DN, 5.0, 1e-3)
    assert e.value.code == -1 and "normals" in str(e.value)
