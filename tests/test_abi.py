"""The C-ABI library loads and exports every symbol include/ffm.h declares (no GPU needed).

Also checks that the host-side argument validation rejects bad calls before touching a device.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "ffm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ffm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    import paper_1909_05600_amd as ffm
    if not os.path.exists(ffm.LIB_PATH):
        from paper_1909_05600_amd import build
        build.build()
    return ffm.lib()


def test_every_declared_symbol_is_exported(L):
    import paper_1909_05600_amd as ffm
    decl = _declared_functions()
    assert set(decl) == set(ffm.EXPORTED), decl
    for name in decl:
        assert hasattr(L, name), name


def test_version_and_last_error(L):
    assert L.ffm_version().decode().startswith("ffm-gfx950")
    assert L.ffm_last_error() is not None


def test_invalid_arguments_are_rejected_before_any_device_work(L):
    import paper_1909_05600_amd as ffm
    h = C.c_void_p()
    dummy = C.c_void_p(0x1000)   # never dereferenced: every call below fails validation first
    cases = [
        (dummy, 10, dummy, 10, 0, 0.0, 1e-3, None, None, None),         # out == NULL
        (dummy, -1, dummy, 10, 0, 0.0, 1e-3, None, None, C.byref(h)),   # negative size
        (None, 10, dummy, 10, 0, 0.0, 1e-3, None, None, C.byref(h)),    # NULL X
        (dummy, 10, dummy, 10, 8, 0.0, 1e-3, None, None, C.byref(h)),   # unknown kernel
        (dummy, 10, dummy, 10, -1, 0.0, 1e-3, None, None, C.byref(h)),  # unknown kernel
        (dummy, 10, dummy, 10, 1, -2.0, 1e-3, None, None, C.byref(h)),  # k < 0
        (dummy, 10, dummy, 10, 1, float("nan"), 1e-3, None, None, C.byref(h)),
        (dummy, 10, dummy, 10, 0, 0.0, 0.0, None, None, C.byref(h)),    # eps <= 0
        (dummy, 10, dummy, 10, 0, 0.0, 1e-9, None, None, C.byref(h)),   # eps too small
        (dummy, 10, dummy, 10, 0, 0.0, 0.7, None, None, C.byref(h)),    # eps too large
        (dummy, 1 << 31, dummy, 10, 0, 0.0, 1e-3, None, None, C.byref(h)),
        (dummy, 10, dummy, 10, 2, 0.0, 1e-3, None, None, C.byref(h)),   # _DN without target normals
        (dummy, 10, dummy, 10, 5, 3.0, 1e-3, None, None, C.byref(h)),   # _DL without source normals
    ]
    for args in cases:
        assert L.ffm_plan(*args) == -1, args
        assert L.ffm_last_error().decode() != ""
    bad = ffm.Options(0, 0, 0.0, 0, 0, 64)      # unknown flag bits
    assert L.ffm_plan(dummy, 10, dummy, 10, 0, 0.0, 1e-3, C.byref(bad), None, C.byref(h)) == -1
    bad = ffm.Options(0, 0, 0.0, 0, 0, 24)      # ACA both forbidden and forced
    assert L.ffm_plan(dummy, 10, dummy, 10, 0, 0.0, 1e-3, C.byref(bad), None, C.byref(h)) == -1
    bad = ffm.Options(0, 0, 0.0, 0, 0, 6)       # direct and grid transforms both forced
    assert L.ffm_plan(dummy, 10, dummy, 10, 0, 0.0, 1e-3, C.byref(bad), None, C.byref(h)) == -1
    bad = ffm.Options(0, 5, 0.0, 0, 0, 0)       # unknown precision
    assert L.ffm_plan(dummy, 10, dummy, 10, 0, 0.0, 1e-3, C.byref(bad), None, C.byref(h)) == -1
    bad = ffm.Options(0, 0, 0.0, 0, 25, 0)      # depth cap above 20
    assert L.ffm_plan(dummy, 10, dummy, 10, 0, 0.0, 1e-3, C.byref(bad), None, C.byref(h)) == -1
    bad = ffm.Options(0, 0, 0.0, 0, 0, 0)       # target normals do not stand in for source normals
    bad.target_normals = dummy.value
    assert L.ffm_plan(dummy, 10, dummy, 10, 4, 0.0, 1e-3, C.byref(bad), None, C.byref(h)) == -1
    assert "source_normals" in L.ffm_last_error().decode()
    assert L.ffm_apply(None, dummy, 0, dummy, None) == -1
    assert L.ffm_destroy(None) == 0
    assert L.ffm_plan_stats(None, None) == -1
    cnt = C.c_int64()
    assert L.ffm_plan_export(None, 0, 0, 0, None, C.byref(cnt)) == -1


def test_batch_arguments_are_rejected_before_any_device_work(L):
    import paper_1909_05600_amd as ffm
    h = C.c_void_p()
    arr = (C.c_void_p * 2)(None, None)
    assert L.ffm_batch_create(arr, 2, 0, None, None, None) == -1          # out == NULL
    assert L.ffm_batch_create(None, 2, 0, None, None, C.byref(h)) == -1   # no plans
    assert L.ffm_batch_create(arr, 0, 0, None, None, C.byref(h)) == -1    # n <= 0
    assert L.ffm_batch_create(arr, 2, 0, None, None, C.byref(h)) == -1    # NULL plan
    assert L.ffm_batch_create(arr, 2, 8, None, None, C.byref(h)) == -1    # unknown flag
    assert h.value is None
    assert L.ffm_batch_apply(None, None, None, None, None) == -1
    ptrs = (C.c_void_p * 2)(None, None)
    assert L.ffm_apply_batched(None, ptrs, ptrs, 2, None) == -1           # no plans
    assert L.ffm_apply_batched(arr, ptrs, ptrs, 0, None) == -1            # n <= 0
    assert L.ffm_apply_batched(arr, ptrs, ptrs, 2, None) == -1            # NULL plan
    assert L.ffm_batch_info(None, None) == -1
    assert L.ffm_batch_destroy(None) == 0
    t = ffm.Tiles(4, 2)
    assert L.ffm_plan_set_tiles(None, C.byref(t), None) == -1
    assert L.ffm_plan_get_tiles(None, C.byref(t)) == -1
    assert "batch" in L.ffm_last_error().decode() or "tiles" in L.ffm_last_error().decode()


def test_server_arguments_are_rejected_before_any_device_work(L):
    import paper_1909_05600_amd as ffm
    h = C.c_void_p()
    assert L.ffm_server_create(None, None) == -1                                    # out == NULL
    for bad in (ffm.ServerOptions(-1, 0, 0.0), ffm.ServerOptions(17, 0, 0.0), ffm.ServerOptions(2, 1, 0.0),
                ffm.ServerOptions(2, 0, -5.0), ffm.ServerOptions(2, 0, float("nan"))):
        assert L.ffm_server_create(C.byref(bad), C.byref(h)) == -1
    assert h.value is None
    t = C.c_int64()
    assert L.ffm_server_submit(None, None, None, 0, None, None, C.byref(t)) == -1
    assert L.ffm_server_wait(None, 1, None) == -1
    d = C.c_int32()
    assert L.ffm_server_poll(None, 1, C.byref(d)) == -1
    assert L.ffm_server_stats(None, None) == -1
    assert L.ffm_server_destroy(None) == 0


def test_oracle_is_not_linked_into_the_product():
    """The GPU library and its binding never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1909_05600_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), os.path.join(dirpath, f)


def test_kernel_names_and_launch_timing_validation(L):
    """Launch records name their kernels as profilers print them; bad timing calls are rejected."""
    import paper_1909_05600_amd as ffm
    # (kernel id, variants) -> symbol, ids in the library's launch order of kinds
    assert ffm.kernel_name(0) == "k_perm_in"
    assert ffm.kernel_name(3, 4, 0) == "k_pw_forward_rings<4, false>"
    assert ffm.kernel_name(7, 2, 1) == "k_pw_backward_rings<2, 2, true, 256>"
    assert ffm.kernel_name(7, 102, 0) == "k_pw_backward_rings<2, 2, false, 128>"
    assert ffm.kernel_name(12, 0, 1) == "k_near<true, false>"
    assert ffm.kernel_name(12, 1, 1) == "k_near<true, true>"
    assert ffm.kernel_name(12, 1, 0) == "k_near<false, false>"
    assert ffm.kernel_name(18, 4, 0) == "k_grid_phi_s<4>"
    assert ffm.kernel_name(18, 0, 0) == "k_grid_phi"
    assert ffm.kernel_name(16, 8, 0) == "k_grid_spread<8>"
    assert ffm.FFM_LAPLACE_GRAD == 6 and ffm.FFM_HELMHOLTZ_GRAD == 7
    assert ffm.kernel_name(28, 1, 1) == "k_near_dl<true, true>"
    assert ffm.kernel_name(29) == "k_lag_anterp_dl"
    assert ffm.kernel_name(34, 0, 1) == "k_near_grad<true, false>"
    assert ffm.kernel_name(26, 0, 1) == "k_near_sym<true, false>"
    assert ffm.kernel_name(26, 7, 1) == "k_near_sym_d<true, true, 3>"
    assert ffm.kernel_name(26, 2, 0) == "k_near_sym_d<false, false, 1>"
    assert ffm.kernel_name(30, 101, 0) == "k_pw_forward_dl<1, 64, false>"
    assert ffm.kernel_name(30, 4, 1) == "k_pw_forward_dl<4, 256, true>"
    buf = C.create_string_buffer(6)
    assert L.ffm_kernel_name(18, 4, 0, buf, 6) == len("k_grid_phi_s<4>")
    assert buf.value == b"k_gri"                       # cut to fit, NUL-terminated
    assert L.ffm_kernel_name(999, 0, 0, None, 0) == -1
    n = C.c_int32(0)
    assert L.ffm_plan_launch_timing(None, None, 0, C.byref(n)) == -1
