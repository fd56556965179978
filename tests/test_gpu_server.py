"""Serving: resident plans, HBM-budget admission, overlapping requests (ffm_server_*).

Each request must give bitwise what its plan's own apply gives (same kernels and work items, a
workspace of its own), alone or in a mix with other requests running at the same time; the budget
must bound the workspace held by running requests; dependent sessions (u_{m+1} = v_m / |v_m|, as in an
iterative solve) driven from several host threads must reproduce their sequential results.
"""
import threading

import numpy as np
import pytest

import ffm_workloads as W
from gpu_common import gpu_plan

pytestmark = pytest.mark.gpu


def _plans():
    import torch
    specs = []
    for w in W.serving_plans(6, seed=5, n_min=5000, n_max=60000):
        specs.append((w.X, w.kernel, w.k, w.eps, {}, w.wu))
    l = W.laplace_sphere(20000, seed=8)
    specs.append((l.X, 0, 0.0, 1e-4, {"precision": 1}, l.wu.astype(np.complex64)))
    g = W.helmholtz_sphere(30000, seed=10, k=60.0)
    specs.append((g.X, 1, g.k, g.eps, {"transforms": "grid"}, g.wu))     # grid-form levels
    plans, wus = [], []
    for X, kern, k, eps, kw, wu in specs:
        plans.append(gpu_plan(X, X, kern, k, eps, **kw))
        wus.append(torch.from_numpy(np.ascontiguousarray(wu)).cuda())
    return plans, wus


def _alone(p, wu):
    import torch
    v = p.apply(wu)
    torch.cuda.synchronize()
    return v.cpu().numpy()


def test_mixed_requests_equal_standalone():
    import torch
    import paper_1909_05600_amd as ffm
    plans, wus = _plans()
    srv = ffm.Server(slots=4)
    reqs = []
    for rep in range(3):                       # three requests per plan, all submitted at once
        for i, (p, w) in enumerate(zip(plans, wus)):
            # wr is written on the current stream; submit orders the request after it (a device-side wait on
            # an event recorded at submission), with no host synchronisation in between
            wr = w * (1.0 + rep)
            t, out = srv.submit(p, wr)
            reqs.append((i, wr, t, out))
    torch.cuda.synchronize()
    lat = [srv.wait(t) for _, _, t, _ in reqs]
    st = srv.stats()
    print("server stats:", st)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["peak_running"] >= 2              # requests overlapped on the device
    assert all(x > 0 for x in lat)
    for i, wr, t, out in reqs:
        assert np.array_equal(out.cpu().numpy(), _alone(plans[i], wr)), i
    srv.destroy()
    for p in plans:
        p.destroy()


def test_budget_bounds_running_workspace():
    import torch
    import paper_1909_05600_amd as ffm
    plans, wus = _plans()
    sizes = [p.stats()["workspace_bytes"] for p in plans]
    budget = 1.2 * max(sizes)
    srv = ffm.Server(slots=4, budget_bytes=budget)
    reqs = [(i,) + srv.submit(p, w) for i, (p, w) in enumerate(zip(plans, wus)) for _ in range(2)]
    for _, t, _ in reqs:
        srv.wait(t)
    st = srv.stats()
    print("budget %.0f: peak in use %.0f, peak running %d" % (budget, st["peak_in_use_bytes"], st["peak_running"]))
    assert 0 < st["peak_in_use_bytes"] <= budget
    for i, t, out in reqs:
        assert np.array_equal(out.cpu().numpy(), _alone(plans[i], wus[i])), i
    # a request whose workspace exceeds the whole budget is refused at submission
    small = ffm.Server(slots=2, budget_bytes=min(sizes) / 2)
    with pytest.raises(ffm.FFMError) as e:
        small.submit(plans[0], wus[0])
    assert e.value.code == -2
    small.destroy()
    # a plan with pending requests cannot be destroyed
    t, _ = srv.submit(plans[1], wus[1])
    try:
        with pytest.raises(ffm.FFMError) as e:
            plans[1].destroy()
        assert e.value.code == -4
    finally:
        srv.wait(t)
    srv.destroy()
    for p in plans:
        p.destroy()


def test_dependent_sessions_from_threads():
    """Sessions of dependent matvecs from concurrent host threads equal the same sessions run one after another."""
    import torch
    import paper_1909_05600_amd as ffm
    plans, wus = _plans()
    steps = 6

    def session(apply_fn, p, w):
        u = w
        hist = []
        for _ in range(steps):
            v = apply_fn(p, u)
            hist.append(v.cpu().numpy())
            u = (v / torch.linalg.vector_norm(v)).contiguous()
            torch.cuda.current_stream().synchronize()
        return hist

    ref = [session(lambda p, u: (p.apply(u), torch.cuda.synchronize())[0], p, w) for p, w in zip(plans, wus)]
    srv = ffm.Server(slots=4)

    def via_server(p, u):
        t, out = srv.submit(p, u)
        srv.wait(t)
        return out

    got = [None] * len(plans)

    def run(i):
        got[i] = session(via_server, plans[i], wus[i])

    ths = [threading.Thread(target=run, args=(i,)) for i in range(len(plans))]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    st = srv.stats()
    print("sessions:", st)
    assert st["completed"] == steps * len(plans)
    for i in range(len(plans)):
        for m in range(steps):
            assert np.array_equal(got[i][m], ref[i][m]), (i, m)
    srv.destroy()
    for p in plans:
        p.destroy()
