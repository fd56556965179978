"""Allocation failure: with FFM_TEST_FAIL_ALLOC_AFTER=n the library refuses the (n+1)-th device allocation of the
process (that one only).  In a child process per n, a plan whose build meets the refusal must return FFM_ENOMEM
and leave no device memory allocated (ffm_device_bytes_live back to zero), and the next plan of the same
workload must build and give bitwise the product of a third, independent plan.  The failure is forced from the
host (the allocation is refused before any device call), so no kernel sees an invalid buffer."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r"""
import json, sys
import numpy as np, torch
sys.path.insert(0, %(root)r)
import ffm_workloads as W
import paper_1909_05600_amd as ffm
w = W.helmholtz_sphere(20000, seed=3, k=40.0)
X = torch.from_numpy(w.X).cuda()
wu = torch.from_numpy(w.wu).cuda()
torch.cuda.synchronize()
out = {"live0": ffm.device_bytes_live()}
try:
    p = ffm.Plan(X, X, ffm.FFM_HELMHOLTZ, w.k, w.eps)
    out["first"] = "ok"
    p.destroy()
except ffm.FFMError as e:
    out["first"] = "enomem" if e.code == -2 else "error %%d" %% e.code
torch.cuda.synchronize()
out["live_after"] = ffm.device_bytes_live()
p2 = ffm.Plan(X, X, ffm.FFM_HELMHOLTZ, w.k, w.eps)
p3 = ffm.Plan(X, X, ffm.FFM_HELMHOLTZ, w.k, w.eps)
v2 = p2.apply(wu).cpu().numpy()
v3 = p3.apply(wu).cpu().numpy()
out["equal"] = bool(np.array_equal(v2, v3))
out["finite"] = bool(np.isfinite(v2).all())
p2.destroy(); p3.destroy()
torch.cuda.synchronize()
out["live_end"] = ffm.device_bytes_live()
print("RESULT " + json.dumps(out), flush=True)
"""


def _run(n):
    env = dict(os.environ, FFM_TEST_FAIL_ALLOC_AFTER=str(n))
    print("child with FFM_TEST_FAIL_ALLOC_AFTER=%d" % n, flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD % {"root": ROOT}], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-3000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


def test_allocation_failure_rolls_back_and_recovers():
    failed = 0
    for n in (0, 4, 25, 60):
        res = _run(n)
        print(n, res)
        assert res["live0"] == 0
        assert res["first"] in ("ok", "enomem"), res
        if res["first"] == "enomem":
            failed += 1
            assert res["live_after"] == 0, res       # nothing of the failed plan stays allocated
        assert res["equal"] and res["finite"], res
        assert res["live_end"] == 0, res
    assert failed >= 3      # the refusals at 0, 4 and 25 fall inside the first plan's build
