#!/usr/bin/env python3
"""FFM throughput on one MI355X.

One step is one complete FFM product v = G W u on the resident synthetic workload
(N = 1,048,576 random points on the unit sphere, sources = targets, Helmholtz kernel,
k for ten points per wavelength, eps = 1e-3): ffm_plan (root cubes, Morton keys, sort,
level boxes, descent lists, transfer tables) + ffm_apply (per-level transforms and transfers,
near field, permutations) + ffm_destroy.  Inputs are in HBM before the timed region.

Prints ONE JSON line (rank 0): points/s of the whole product, apply-only points/s, the roofline of
the dominant kernel measured live with the library's HIP events on the apply stream, and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz = 39.3e12 VALU issue slots/s (FP32 non-packed,
# the form this library is built for); reported as FMA-equivalent TFLOP/s = 2 x slots/s.
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
PEAK_ALU_TFLOPS = 2 * VALU_SLOTS_PER_S / 1e12          # 78.6
# Minimal non-transcendental VALU slots of the plane-wave transforms as implemented (sin/cos run on the
# transcendental unit at half rate, co-issued, and take FP32 phases unreduced; see profiles/peaks_mi355x.txt):
#   direction-pair form: per (point, antipodal pair)   3 phase + 4 accumulate = 7 slots / 2 directions
#   ring-pair form:      per (point, group of 4 dirs)   2 phase + 8 accumulate = 10 slots / 4 directions
SLOTS_PER_DIRECTION = {1: 7 / 2, 2: 10 / 4}
# Near field, per (target, source) pair: Laplace ~10 non-transcendental slots, Helmholtz ~18 (plus sin, cos and
# reciprocal square root on the transcendental unit).
NEAR_SLOTS = {"k_near<false>": 10.0, "k_near<true>": 18.0}
# Published MI355X peaks per bound: dense FP32 MFMA 157.3 TFLOP/s, FP32 VALU (non-packed, FMA = 2) 78.6,
# HBM3E 8 TB/s.
PEAKS = {"mfma": (157.3, "TFLOP/s"), "alu": (PEAK_ALU_TFLOPS, "TFLOP/s"), "hbm": (8000.0, "GB/s")}

# HBM traffic per launch of the dominant kernel from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of this
# workload (profiles/traffic_apply_helmholtz_sphere_1M.md), scaled by what the counters read for a copy
# kernel of known size (FETCH x 2.0, WRITE x 1.0), mean over the kernel's launches in one product.  Valid only
# for the kernel source it was taken on.
TRAFFIC_SOURCE_HASH = "d19c06e41360a2d6"      # sha256 prefix of paper_1909_05600_amd/csrc/apply.hip
TRAFFIC = {
    "k_near<true>": (382161.0 * 2.0 + 8833.875) * 1024.0,
    "k_grid_phit": (79074.875 * 2.0 + 295680.0) * 1024.0,
}


def _source_hash():
    import hashlib
    with open(os.path.join(ROOT, "paper_1909_05600_amd", "csrc", "apply.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-strides", type=str, default="64,128")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-instance batched workload")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving workload")
    ap.add_argument("--serving-matvecs", type=int, default=10,
                    help="dependent matvecs per session in the serving workload (50 in the full study)")
    ap.add_argument("--serving-loads", type=str, default="0.8",
                    help="offered loads as fractions of the one-at-a-time capacity, e.g. 0.5,0.8,0.95")
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--mixed-study", action="store_true",
                    help="only run the 10M-point sphere + cube study (FP32 and mixed precision at eps 1e-3, 1e-4)")
    ap.add_argument("--mixed-n", type=int, default=10_000_000)
    ap.add_argument("--bie-study", action="store_true",
                    help="only run the single-layer sphere solve (GMRES with FFM products) at --bie-n nodes")
    ap.add_argument("--bie-n", type=int, default=1 << 20)
    ap.add_argument("--bie-eps", type=float, default=1e-3)
    ap.add_argument("--bie-tol", type=float, default=1e-4)
    ap.add_argument("--mixed-rows", type=int, default=1024)
    return ap.parse_args()


def cpu_baseline(w, strides):
    """The FP64 oracle as it stands, on the host cores: full tree and lists, then the per-box loops of
    every level (transforms, transfers, near field) on every s-th box for two strides s; the time of the
    full product is a + b with t(s) = a + b / s fitted through the two samples."""
    import oracle
    t0 = time.perf_counter()
    p = oracle.Plan(w.X, w.X, w.kernel, w.k, w.eps)
    t_plan = time.perf_counter() - t0
    ts = []
    for s in strides:
        t0 = time.perf_counter()
        p.apply(w.wu, stride=s)
        ts.append(time.perf_counter() - t0)
    (s1, s2), (t1, t2) = strides, ts
    b = (t1 - t2) / (1.0 / s1 - 1.0 / s2)
    a = t1 - b / s1
    if b <= 0:          # degenerate fit: fall back to scaling the larger sample
        a, b = 0.0, t1 * s1
    t_full = t_plan + max(a, 0.0) + b
    return {
        "value": w.n / t_full, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
        "sample": "FP64 oracle FFM at N=%d: full tree/lists (%.1fs), per-box loops on every %d-th and "
                  "every %d-th box (%.1fs, %.1fs); full product time a + b from t(s) = a + b/s, est. %.0fs"
                  % (w.n, t_plan, s1, s2, t1, t2, t_full),
    }


def dense_rows_device(X, wu, kernel, k, rows, chunk=1 << 15):
    """FP64 direct sums v_i = sum_{j: r_ij > 0} G(x_i, x_j) wu_j on sampled target rows, in plain torch on the
    device (the reference for the error figures; sources = targets = X, G = e^{ikr}/(4 pi r) or 1/(4 pi r))."""
    import torch
    R = X[torch.as_tensor(np.asarray(rows, dtype=np.int64), device=X.device)]
    u = wu.to(torch.complex128)
    acc = torch.zeros(R.shape[0], dtype=torch.complex128, device=X.device)
    for s in range(0, X.shape[0], chunk):
        d = R[:, None, :] - X[None, s:s + chunk, :]
        r = torch.sqrt((d * d).sum(-1))
        inv = torch.where(r > 0, 1.0 / (4.0 * math.pi * r), torch.zeros_like(r))
        g = torch.polar(inv, k * r) if kernel == 1 else inv.to(torch.complex128)
        acc += g @ u[s:s + chunk]
    return acc.cpu().numpy()


def _sync_time(fn, reps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def batched(reps=5):
    """256 independent instances (N log-uniform in [2e3, 2e5], half Laplace / half Helmholtz, sphere /
    ellipsoid / cube; resident plans): apply points/s of (a) one ffm_apply per instance in FP32, (b) the
    FP32 batch replayed from a HIP graph with autotuned tiles, (c) the same with mixed-precision plans
    (FP16 MFMA transfers on Lagrange levels); accuracy of (b) and (c) against FP64 dense rows (16 sampled
    targets per instance)."""
    import torch
    import ffm_workloads as W
    import paper_1909_05600_amd as ffm
    ws = W.batched_instances(256, seed=4)
    n_tot = sum(w.n for w in ws)
    Xs = [torch.from_numpy(w.X).cuda() for w in ws]
    wus = [torch.from_numpy(w.wu).cuda() for w in ws]
    outs = [torch.empty(w.n, dtype=torch.complex64, device="cuda") for w in ws]
    res = {"instances": len(ws), "points": n_tot}
    t0 = time.perf_counter()
    p32 = [ffm.Plan(X, X, w.kernel, w.k, w.eps) for X, w in zip(Xs, ws)]
    torch.cuda.synchronize()
    res["plan_s_fp32"] = time.perf_counter() - t0
    pmx = [ffm.Plan(X, X, w.kernel, w.k, w.eps, precision=ffm.FFM_PREC_MIXED) for X, w in zip(Xs, ws)]

    def single():
        for p, u, o in zip(p32, wus, outs):
            p.apply(u, out=o)

    single()
    t = _sync_time(single, reps)
    res["fp32_per_instance_points_per_s"] = n_tot / t
    res["fp32_per_instance_ms"] = t * 1e3
    for name, plans in (("fp32_batched_graph", p32), ("mixed_batched_graph", pmx)):
        b = ffm.Batch(plans, graph=True, autotune=True)
        o2 = [torch.empty_like(o) for o in outs]
        b.apply(wus, outs=o2)
        t = _sync_time(lambda: b.apply(wus, outs=o2), reps)
        info = b.info()
        errs = []
        for w, X, u, o in zip(ws, Xs, wus, o2):
            rows = w.rows[:16]
            d = dense_rows_device(X, u, w.kernel, w.k, rows)
            v = o.cpu().numpy()[rows].astype(np.complex128)
            errs.append(float(np.linalg.norm(v - d) / np.linalg.norm(d)))
        res[name + "_points_per_s"] = n_tot / t
        res[name + "_ms"] = t * 1e3
        res[name + "_launches"] = info["launches"]
        res[name + "_tiles"] = list(info["tiles"])
        res[name + "_err_max"] = max(errs)
        res[name + "_err_median"] = float(np.median(errs))
        b.destroy()
    for p in p32 + pmx:
        p.destroy()
    res["eps"] = ws[0].eps
    return res


def serving(matvecs, loads, slots):
    """64 resident plans (N log-uniform in [1e4, 5e6], Laplace / Helmholtz alternating, 10 points per
    wavelength, sphere / ellipsoid / cube); a session is `matvecs` dependent applies u_{m+1} = v_m/|v_m|;
    sessions start at Poisson times at a given fraction of the one-at-a-time capacity.  The same arrival
    trace runs through the server with `slots` concurrent slots and through a one-slot server (requests
    one at a time, in arrival order).  Reports points/s over the makespan and p50/p99 request latency
    (submission to completion)."""
    import torch
    import ffm_workloads as W
    import paper_1909_05600_amd as ffm
    ws = W.serving_plans(64, seed=5)
    plans, u0 = [], []
    for w in ws:
        X = torch.from_numpy(w.X).cuda()
        plans.append(ffm.Plan(X, X, w.kernel, w.k, w.eps))
        u0.append(torch.from_numpy(w.wu).cuda())
        del X
    torch.cuda.synchronize()
    # one-at-a-time service time of a session -> capacity in sessions/s
    t_apply = []
    for p, u in zip(plans, u0):
        p.apply(u)
        t_apply.append(_sync_time(lambda: p.apply(u), 1))
    t_session = matvecs * float(np.mean(t_apply))
    out = {"plans": len(plans), "points_per_request_mean": float(np.mean([w.n for w in ws])),
           "matvecs_per_session": matvecs, "session_s_one_at_a_time": t_session, "loads": []}
    norm_stream = torch.cuda.Stream()

    def run(rate, nslots):
        arr = W.poisson_arrivals(len(plans), rate, seed=5)
        srv = ffm.Server(slots=nslots)
        state = [None] * len(plans)       # (ticket, out, step)
        lat = []
        started = done = 0
        total_pts = 0.0
        t0 = time.perf_counter()
        while done < len(plans):
            now = time.perf_counter() - t0
            progressed = False
            while started < len(plans) and arr[started] <= now:
                t, o = srv.submit(plans[started], u0[started])
                state[started] = (t, o, 0)
                started += 1
                progressed = True
            for i in range(started):
                st = state[i]
                if st is None or not srv.poll(st[0]):
                    continue
                lat.append(srv.wait(st[0]))
                total_pts += plans[i].n_x
                step = st[2] + 1
                progressed = True
                if step == matvecs:
                    state[i] = None
                    done += 1
                    if done % 8 == 0:
                        print("serving: %d-slot run, %d of %d sessions done" % (nslots, done, len(plans)),
                              file=sys.stderr, flush=True)
                    continue
                with torch.cuda.stream(norm_stream):
                    v = st[1]
                    u = (v / torch.linalg.vector_norm(v)).contiguous()
                norm_stream.synchronize()
                t, o = srv.submit(plans[i], u)
                state[i] = (t, o, step)
            if not progressed:
                time.sleep(50e-6)
        makespan = time.perf_counter() - t0
        srv.destroy()
        return {"points_per_s": total_pts / makespan, "makespan_s": makespan,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "requests": len(lat)}

    for rho in loads:
        rate = rho / t_session
        served = run(rate, slots)
        fifo = run(rate, 1)
        out["loads"].append({"load": rho, "sessions_per_s": rate, "server": served, "one_at_a_time": fifo,
                             "slots": slots})
        print("serving load %.2f: %d-slot %.3g pts/s p50 %.1f ms p99 %.1f ms | one-at-a-time %.3g pts/s "
              "p50 %.1f ms p99 %.1f ms" % (rho, slots, served["points_per_s"], served["p50_ms"],
                                          served["p99_ms"], fifo["points_per_s"], fifo["p50_ms"],
                                          fifo["p99_ms"]), file=sys.stderr, flush=True)
    for p in plans:
        p.destroy()
    return out


def mixed_study(n, n_rows, reps=3):
    """Helmholtz on 80% sphere + 20% cube cluster points (non-uniform octree), k by ten points per wavelength
    on the sphere: plan and apply time per precision mode and eps, and the error against FP64 dense rows on
    sampled targets, overall and per target class (sphere / cube)."""
    import torch
    import ffm_workloads as W
    import paper_1909_05600_amd as ffm
    out = {"n": n, "rows": n_rows, "runs": []}
    w = W.sphere_plus_cube(n, seed=3, n_rows=n_rows)     # the points, u and rows do not depend on eps
    out["k"] = w.k
    X = torch.from_numpy(w.X).cuda()
    wu = torch.from_numpy(w.wu).cuda()
    t0 = time.perf_counter()
    d = dense_rows_device(X, wu, 1, w.k, w.rows)
    t_dense = time.perf_counter() - t0
    sph = w.rows < w.meta["n_sphere"]
    for eps in (1e-3, 1e-4):
        for prec in (0, 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p = ffm.Plan(X, X, 1, w.k, eps, precision=prec)
            torch.cuda.synchronize()
            t_plan = time.perf_counter() - t0
            v = p.apply(wu)
            t_apply = _sync_time(lambda: p.apply(wu, out=v), reps)
            vv = v.cpu().numpy()[w.rows].astype(np.complex128)
            st = p.stats()

            def rl(a, b):
                return float(np.linalg.norm(a - b) / np.linalg.norm(b))
            r = {"eps": eps, "precision": "mixed" if prec else "fp32", "plan_s": t_plan, "apply_s": t_apply,
                 "points_per_s": n / (t_plan + t_apply), "apply_points_per_s": n / t_apply,
                 "err": rl(vv, d), "err_sphere": rl(vv[sph], d[sph]), "err_cube": rl(vv[~sph], d[~sph]),
                 "leaf": st["leaf"], "methods": st["method"][:st["leaf"] + 1],
                 "fp16_levels": [l for l in range(st["leaf"] + 1) if st["prec"][l]],
                 "phase64_levels": [l for l in range(st["leaf"] + 1) if st["phase64"][l]],
                 "plan_mb": st["plan_bytes"] / 1e6, "workspace_mb": st["workspace_bytes"] / 1e6,
                 "dense_rows_s": t_dense}
            out["runs"].append(r)
            print("mixed study eps=%g %s: plan %.2fs apply %.3fs err %.2e (sphere %.2e cube %.2e)"
                  % (eps, r["precision"], t_plan, t_apply, r["err"], r["err_sphere"], r["err_cube"]),
                  file=sys.stderr, flush=True)
            p.destroy()
            torch.cuda.empty_cache()
    return out


def bie_study(n, eps, tol, kernels=(0, 1)):
    """The single-layer equation on the unit sphere (reduced Gauss grid with about n nodes): GMRES with one FFM
    product per iteration, for Laplace (data: the potential of a point charge inside the sphere) and for
    Helmholtz at ten nodes per wavelength (data: a plane wave on a sound-soft sphere).
    Reports set-up (plan + the correction's product), iterations, solve time, products per second and the
    error of the density against the closed form (harmonics divided by their eigenvalues)."""
    import torch
    import ffm_workloads as W
    from paper_1909_05600_amd import bie
    out = {"n_target": n, "eps": eps, "tol": tol, "runs": []}
    for kernel in kernels:
        p = W.bie_sphere(W.n_theta_for(n), kernel, None, eps, data="source" if kernel == 0 else "plane_wave")
        X = torch.from_numpy(p.X).cuda()
        w = torch.from_numpy(p.w).cuda()
        f = torch.from_numpy(p.f).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A = bie.SingleLayer(X, w, kernel, p.k, eps)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        bie.solve(A, f, tol=0.5, restart=100, maxiter=1)   # warms up the library kernels and the basis memory
        A.products = 1
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sigma, info = bie.solve(A, f, tol=tol, restart=100, maxiter=2000)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t0
        if kernel == 0:
            exact = bie.zonal_density(p.X, p.x0, bie.point_source_coefficients(np.linalg.norm(p.x0), p.radius))
        else:
            exact = bie.plane_wave_density(p.X, p.direction, p.k, p.radius)
        s = sigma.cpu().numpy().astype(np.complex128)
        sw = np.sqrt(p.w)
        err = float(np.linalg.norm((s - exact) * sw) / np.linalg.norm(exact * sw))
        res = float(torch.linalg.vector_norm(A.matvec(sigma) - f.to(torch.complex64))
                    / torch.linalg.vector_norm(f))
        st = A.plan.stats()
        t_mv = _sync_time(lambda: A.matvec(sigma), 5)
        r = {"kernel": "laplace" if kernel == 0 else "helmholtz", "data": p.data, "n": p.n, "k": p.k, "setup_s": t_setup,
             "solve_s": t_solve, "iterations": info["iterations"], "converged": info["converged"],
             "products": A.products - 1, "ms_per_iteration": t_solve * 1e3 / max(1, info["iterations"]),
             "matvec_ms": t_mv * 1e3, "final_residual": res, "err_vs_closed_form": err, "leaf": st["leaf"],
             "transform_form": [int(x) for x in st["tform"][:st["leaf"] + 1]]}
        out["runs"].append(r)
        print("bie study %s N=%d k=%.2f: setup %.3fs, %d iterations in %.3fs (%.2f ms each, matvec %.2f ms), "
              "residual %.2e, error vs closed form %.2e" % (r["kernel"], p.n, p.k, t_setup, r["iterations"],
                                                            t_solve, r["ms_per_iteration"], t_mv * 1e3, res, err),
              file=sys.stderr, flush=True)
        A.destroy()
        del X, w, f, sigma
        torch.cuda.empty_cache()
    return out


def kernel_totals(launches, steps):
    """Milliseconds per step of every kernel symbol over the timed steps (HIP events around each launch)."""
    tot = {}
    for step in launches:
        for r in step:
            tot[r["kernel"]] = tot.get(r["kernel"], 0.0) + r["ms"] / steps
    return dict(sorted(tot.items(), key=lambda kv: -kv[1]))


def launch_work(name, level, st):
    """Algorithmic work of one launch of a kernel at a level: (amount, unit kind, definition), or None for
    kernels without a model here.  mfma / alu amounts are flops (FMA = 2), hbm amounts bytes."""
    L, nq = st["order"][level], st["nq"][level]
    p, nbf, nbt = st["grid_nodes"][level], st["fwd_boxes"][level], st["bwd_boxes"][level]
    if name.startswith("k_grid_phi"):
        nb = nbt if name == "k_grid_phit" else nbf
        return (8.0 * nb * (L + 1) * p * p * L, "mfma",
                "8 flops per (box, ring, node a, node b, azimuth): the four real products of the separable "
                "plane sums, FP32 MFMA")
    if name in ("k_grid_z", "k_grid_zt"):
        nb = nbf if name == "k_grid_z" else nbt
        return (8.0 * nb * ((L + 2) // 2) * p ** 3, "mfma",
                "8 flops per (box, ring pair, plane, column): the four real products of the z sums, FP32 MFMA")
    if name.startswith("k_pw_forward_rings") or name.startswith("k_pw_backward_rings"):
        pts = st["fwd_points"][level] if "forward" in name else st["bwd_points"][level]
        return (2.0 * SLOTS_PER_DIRECTION[2] * pts * nq, "alu",
                "non-transcendental VALU issue slots x 2 of the ring-pair form: 10 per (point, 4 directions)")
    if name.startswith("k_pw_forward") or name.startswith("k_pw_backward"):
        pts = st["fwd_points"][level] if "forward" in name else st["bwd_points"][level]
        return (2.0 * SLOTS_PER_DIRECTION[1] * pts * nq, "alu",
                "non-transcendental VALU issue slots x 2 of the direction-pair form: 7 per (point, 2 directions)")
    if name.startswith("k_near"):
        return (2.0 * NEAR_SLOTS[name] * st["near_pairs"], "alu",
                "non-transcendental VALU issue slots x 2 per (target, source) pair of the near field")
    if name.startswith("k_pw_transfer"):
        return (8.0 * nq * (nbf + st["nclass"][level] + nbt), "hbm",
                "unique bytes: u~ of every source box, the class tables D and v~ of every target box, 8 per "
                "direction each (the far-pair gathers re-read them from the caches)")
    return None


def roofline(launches, st, steps):
    """Roofline of the dominant kernel: the kernel symbol with the most time per step among those with a
    work model; achieved = its algorithmic work over all its launches / their HIP-event time."""
    tot = kernel_totals(launches, steps)
    for name in tot:
        work, kind, definition, ms, n = 0.0, None, None, 0.0, 0
        for step in launches:
            for r in step:
                if r["kernel"] != name:
                    continue
                m = launch_work(name, r["level"], st)
                if m is None:
                    break
                work += m[0]
                kind, definition = m[1], m[2]
                ms += r["ms"]
                n += 1
        if kind is None or ms <= 0:
            continue
        peak, unit = PEAKS[kind]
        rate = work / (ms * 1e-3) / (1e12 if unit == "TFLOP/s" else 1e9)
        return name, {"bound": kind, "kernel": name, "achieved": rate, "peak": peak, "unit": unit,
                      "frac": rate / peak, "launches": n // steps, "avg_launch_ms": ms / n,
                      "work_per_step": work / steps, "work": definition}
    return "none", {"bound": "alu", "kernel": "none", "achieved": 0.0, "peak": PEAK_ALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": 0.0}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported (one GPU per box here)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import ffm_workloads as W
    import paper_1909_05600_amd as ffm

    if args.mixed_study:
        res = {"metric": "10M sphere + cube Helmholtz: points/s and error per precision mode",
               "mixed_study": mixed_study(args.mixed_n, args.mixed_rows)}
        print(json.dumps(res), flush=True)
        return

    if args.bie_study:
        res = {"metric": "single-layer sphere solve: GMRES iterations, time and error vs the closed form",
               "bie_study": bie_study(args.bie_n, args.bie_eps, args.bie_tol)}
        print(json.dumps(res), flush=True)
        return

    w = W.helmholtz_sphere(args.n, seed=2, eps=args.eps)
    dev = torch.device("cuda:0")
    X = torch.from_numpy(w.X).to(dev)
    wu = torch.from_numpy(w.wu).to(dev)
    out = torch.empty(w.n, dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    tiles = [4, 2]
    plan_stream = torch.cuda.Stream()

    def make_plan():
        t0 = time.perf_counter()
        plan = ffm.Plan(X, X, ffm.FFM_HELMHOLTZ, w.k, w.eps, timing=True, stream=plan_stream)
        return plan, t0, time.perf_counter()

    def run(nsteps, record):
        """nsteps complete products; the plan of product i+1 is built (host work, and its kernels on a
        second stream) while product i's apply runs on the GPU, and product i+1's apply is enqueued as soon as
        its plan is complete, before product i's completion is awaited and its plan destroyed: every product
        still runs its own full plan, apply and destroy, and its apply starts only once its plan is complete.
        Latency ends at the apply's end on the GPU clock, mapped to the host clock through a reference event."""
        if nsteps == 0:
            return
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(stream)
        ref.synchronize()
        t_ref = time.perf_counter()

        def finish(ent):
            plan, tp0, tp1, e0, e1 = ent
            e1.synchronize()
            if record is not None:
                t_done = t_ref + ref.elapsed_time(e1) * 1e-3
                record["plan_ms"].append((tp1 - tp0) * 1e3)
                record["apply_ms"].append(e0.elapsed_time(e1))
                record["latency_ms"].append((t_done - tp0) * 1e3)
                record["phases"].append(plan.timing())
                record["launches"].append(plan.launch_timing())
                record["stats"] = plan.stats()
            plan.destroy()

        cur = make_plan()
        prev = None
        for i in range(nsteps):
            plan, tp0, tp1 = cur
            tiles[:] = plan.tiles()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            plan.apply(wu, out=out, stream=stream)
            e1.record(stream)
            if prev is not None:
                finish(prev)
            prev = (plan, tp0, tp1, e0, e1)
            cur = make_plan() if i + 1 < nsteps else None
        finish(prev)

    run(args.warmup, None)
    rec = {"plan_ms": [], "apply_ms": [], "latency_ms": [], "phases": [], "launches": [], "stats": None}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    run(args.steps, rec)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = t_total * 1e3 / args.steps
    step_ms = rec["latency_ms"]

    st = rec["stats"]
    ph = np.array(rec["phases"])          # [steps][64]
    leaf = st["leaf"]
    dom, roof = roofline(rec["launches"], st, args.steps)
    traffic = TRAFFIC.get(dom) if _source_hash() == TRAFFIC_SOURCE_HASH else None
    phase_mean = ph.mean(axis=0)
    names = {0: "perm_in", 61: "near_field", 62: "perm_out"}
    for l in range(1, leaf + 1):
        for j, n in enumerate(("src_transform", "transfer", "tgt_transform")):
            names[1 + 3 * (l - 1) + j] = "l%d_%s" % (l, n)
    phases = {names[i]: round(float(phase_mean[i]), 4) for i in sorted(names) if phase_mean[i] > 0}

    res = {
        "metric": "FFM apply points/s at eps=1e-3 (N=1M Helmholtz) + p50/p99 request latency",
        "value": w.n / (ms_per_step * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "helmholtz_sphere", "n": w.n, "k": round(w.k, 4), "eps": w.eps,
                   "points": "uniform on the unit sphere (seed 2), sources = targets",
                   "u": "complex64, Re/Im ~ N(0,1), w = 4 pi / N",
                   "step": "ffm_plan + ffm_apply + ffm_destroy (the whole product); the plan of the next "
                           "product is built while this product's apply runs, and its apply is enqueued as soon "
                           "as that plan is complete"},
        "apply_points_per_s": w.n / (np.mean(rec["apply_ms"]) * 1e-3),
        "apply_ms": float(np.mean(rec["apply_ms"])),
        "plan_ms": float(np.mean(rec["plan_ms"])),
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "definition": "per product, from the start of its plan to the end of its apply",
                       "per_product": [round(float(x), 3) for x in step_ms]},
        "plan_ms_per_product": [round(float(x), 3) for x in rec["plan_ms"]],
        "plan_plus_apply_ms": float(np.mean(rec["plan_ms"]) + np.mean(rec["apply_ms"])),
        "sequential_points_per_s": w.n / ((np.mean(rec["plan_ms"]) + np.mean(rec["apply_ms"])) * 1e-3),
        "phases_ms": phases,
        "roofline": dict(roof, traffic=traffic,
                         traffic_unit="bytes per launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, factors from a "
                                      "1 GiB copy)"),
        "kernels_ms_per_step": {k: round(v, 4) for k, v in kernel_totals(rec["launches"], args.steps).items()},
        "levels": {"leaf": leaf, "nq": [int(x) for x in st["nq"][:leaf + 1]],
                   "transform_form": [int(x) for x in st["tform"][:leaf + 1]],
                   "grid_nodes": [int(x) for x in st["grid_nodes"][:leaf + 1]],
                   "grid_width": [int(x) for x in st["grid_width"][:leaf + 1]],
                   "nfar": [int(x) for x in st["nfar"][:leaf + 1]], "near_pairs": st["near_pairs"],
                   "transform_terms": st["transform_terms"]},
    }
    del X, wu, out
    torch.cuda.empty_cache()
    if not args.no_batched:
        print("bench: batched workload", file=sys.stderr, flush=True)
        res["batched"] = batched()
        torch.cuda.empty_cache()
    if not args.no_serving:
        print("bench: serving workload", file=sys.stderr, flush=True)
        res["serving"] = serving(args.serving_matvecs, [float(x) for x in args.serving_loads.split(",")],
                                 args.serving_slots)
    if not args.no_cpu_baseline:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        strides = tuple(int(s) for s in args.cpu_strides.split(","))
        res["cpu_baseline"] = cpu_baseline(w, strides)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
