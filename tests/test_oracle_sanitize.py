"""The oracle under host sanitizers: oracle/ffm_oracle.c and a driver (tests/oracle_sanitize.c) built with gcc's
AddressSanitizer and UndefinedBehaviorSanitizer run every oracle entry point on small inputs (both kernels,
Lagrange and Gegenbauer levels, direct and grid transforms, ACA, the normal derivative, the per-pair leaf rule,
distinct and empty sets); any out-of-bounds access, leak or undefined operation aborts it, and its products are
checked against the dense definition."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I" + os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "ffm_oracle.c"),
           os.path.join(HERE, "oracle_sanitize.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "failures 0" in r.stdout
