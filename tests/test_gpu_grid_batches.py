"""Grid form in box batches: the boxes of a grid-form level go through spreading, the z sums and the plane sums
(and on the target side the mirror stages) in batches whose grids G and ring sums H share one workspace slot
range.  The batching changes neither the arithmetic nor any summation order, so a plan whose workspace budget
forces several batches per level (test hook FFM_TEST_GRID_BATCH_BYTES, read once per process) must give
bitwise the product of an unbatched plan, alone and merged with other instances in a batch, with a smaller
workspace."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CHILD = r"""
import hashlib, json, sys
import numpy as np, torch
sys.path.insert(0, %(root)r)
import ffm_workloads as W
import paper_1909_05600_amd as ffm
out = {}
w = W.helmholtz_sphere(60000, seed=11, k=140.0)
X = torch.from_numpy(w.X).cuda()
wu = torch.from_numpy(w.wu).cuda()
p = ffm.Plan(X, X, ffm.FFM_HELMHOLTZ, w.k, w.eps, transforms="grid")
st = p.stats()
out["grid_levels"] = [l for l in range(st["leaf"] + 1) if st["tform"][l] == 3]
out["workspace"] = p.workspace_bytes()
v = p.apply(wu).cpu().numpy()
out["alone"] = hashlib.sha256(v.tobytes()).hexdigest()
# merged with a second instance in a batch (graph replay)
g = W.helmholtz_sphere(20000, seed=12, k=60.0)
Xg = torch.from_numpy(g.X).cuda()
wg = torch.from_numpy(g.wu).cuda()
q = ffm.Plan(Xg, Xg, ffm.FFM_HELMHOLTZ, g.k, g.eps, transforms="grid")
b = ffm.Batch([p, q], graph=True)
outs = b.apply([wu, wg])
torch.cuda.synchronize()
out["batched"] = hashlib.sha256(outs[0].cpu().numpy().tobytes()).hexdigest()
out["batched2"] = hashlib.sha256(outs[1].cpu().numpy().tobytes()).hexdigest()
out["alone2"] = hashlib.sha256(q.apply(wg).cpu().numpy().tobytes()).hexdigest()
b.destroy()
p.destroy()
q.destroy()
print("RESULT " + json.dumps(out), flush=True)
"""


def _run(budget):
    env = dict(os.environ)
    env.pop("FFM_TEST_GRID_BATCH_BYTES", None)
    if budget:
        env["FFM_TEST_GRID_BATCH_BYTES"] = str(budget)
    print("child with grid batch budget %s" % (budget or "default"), flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD % {"root": ROOT}], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-3000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


def test_box_batches_equal_one_batch():
    ref = _run(0)
    small = _run(24 << 20)      # a few boxes per batch at every grid level
    print(ref)
    print(small)
    assert ref["grid_levels"] and ref["grid_levels"] == small["grid_levels"]
    assert small["workspace"] < ref["workspace"]
    assert small["alone"] == ref["alone"]
    assert small["batched"] == ref["batched"] == ref["alone"]
    assert small["batched2"] == ref["batched2"] == ref["alone2"] == small["alone2"]
