"""Helpers shared by the GPU tests: device upload, the HIP plan, comparisons with the oracle."""
import numpy as np

# |v_gpu - v_oracle| / |v_oracle| for the FP32 path against the FP64 oracle with identical parameters: the same
# tree, lists, orders and forms per level, and where a level runs the grid form of the transforms, the same grid
# (p, w, beta; oracle_grid below), so that the two differ by FP32 rounding alone.  The bound is the contract's
# 1e-5 for the FP32 form; the rounding it covers (each stage rounds to 2^-24 and sums random-signed terms, so
# ~sqrt(n) 6e-8 per stage; FP32 phases of up to ~12 revolutions, ~5e-6 rad; the Gegenbauer diagonal's
# cancellation) is derived in the design notes, section 4.
FP32_RTOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def oracle_grid(gp) -> dict:
    """The grid-form parameters (p, w, beta) of every level of a GPU plan that runs the grid form."""
    st = gp.stats()
    return {l: (st["grid_nodes"][l], st["grid_width"][l], st["grid_beta"][l])
            for l in range(1, st["leaf"] + 1) if st["tform"][l] == 3}


def oracle_aca(gp) -> list:
    """The levels of a GPU plan whose transfers use ACA factors (relative tolerance eps / 4)."""
    st = gp.stats()
    return [l for l in range(1, st["leaf"] + 1) if st["aca"][l]]


def oracle_like(orc, gp, X, Y, kernel, k, eps, **kw):
    """The oracle's plan with the GPU plan's parameters (its grid-form and ACA levels included)."""
    return orc.Plan(X, Y, kernel, k, eps, grid=oracle_grid(gp), aca=oracle_aca(gp), aca_tol=eps / 4.0, **kw)


def gpu_plan(X, Y, kernel, k, eps, **kw):
    import torch
    import paper_1909_05600_amd as ffm
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Yd = Xd if Y is X else torch.from_numpy(np.ascontiguousarray(Y)).cuda()
    return ffm.Plan(Xd, Yd, kernel, k, eps, **kw)


def gpu_apply(plan, wu):
    import torch
    v = plan.apply(torch.from_numpy(np.ascontiguousarray(wu)).cuda())
    torch.cuda.synchronize()
    return v.cpu().numpy().astype(np.complex128)


def compare_trees(gp, op, levels=None):
    """Bit-exact comparison of keys, permutation, boxes and descent lists (HIP plan vs oracle plan)."""
    import paper_1909_05600_amd as ffm
    st = gp.stats()
    assert st["leaf"] == op.leaf, (st["leaf"], op.leaf)
    assert st["d0"] == op.d0
    for s in (0, 1):
        assert np.array_equal(np.array(st["corner_x" if s == 0 else "corner_y"]), op.corner(s))
        assert np.array_equal(gp.export(ffm.FFM_EXPORT_KEYS, s), op.keys(s))
        assert np.array_equal(gp.export(ffm.FFM_EXPORT_PERM, s), op.perm(s))
    lv = range(0, op.leaf + 1) if levels is None else levels
    for l in lv:
        for s in (0, 1):
            assert np.array_equal(gp.export(ffm.FFM_EXPORT_BOX_START, s, l), op.box_start(s, l)), (s, l)
            assert np.array_equal(gp.export(ffm.FFM_EXPORT_BOX_IJK, s, l), op.box_ijk(s, l)), (s, l)
            assert np.array_equal(gp.export(ffm.FFM_EXPORT_BOX_CTR, s, l), op.box_centre(s, l)), (s, l)
        if l >= 1:
            t, src, off = op.far(l)
            g = gp.export(ffm.FFM_EXPORT_FAR, 0, l)
            assert np.array_equal(g[:, 0], t) and np.array_equal(g[:, 1], src), l
            assert np.array_equal(g[:, 2:5], off.astype(np.int64)), l
            nt, ns = op.near(l)
            g = gp.export(ffm.FFM_EXPORT_NEAR, 0, l)
            assert np.array_equal(g[:, 0], nt) and np.array_equal(g[:, 1], ns), l
            assert st["method"][l] == op.method(l) and st["order"][l] == op.order(l), l
