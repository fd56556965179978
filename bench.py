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

# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz = 39.3e12 FP32 lane operations/s without packed FP32 (this
# library is built with packed FP32 disabled); an FMA counts 2 flops: 78.6 TFLOP/s.  The data-sheet 157.3 counts
# the packed form and is reported beside it.
VALU_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
PEAK_ALU_TFLOPS = 2 * VALU_SLOTS_PER_S / 1e12          # 78.6
PEAK_ALU_PACKED_TFLOPS = 157.3
# Algorithmic flops (an FMA = 2, a sine, cosine or reciprocal square root = 1):
#   plane-wave transforms in the forms implemented, which share phases between directions by the quadrature's
#   symmetries: the direction-pair form, per (point, antipodal pair): 3 FMA of phase (6) + sin + cos (2) + the
#   two directions' complex multiply-adds from one cos/sin pair (4 FMA, 8): 16 per 2 directions; the ring-pair
#   form, per (point, 4 directions of two mirror rings and two opposite azimuths): 2 FMA of phase (4) + sin +
#   cos (2) + 8 FMA (16): 22 per 4 directions.  (The plain per-term count, 3 FMA of phase + sin + cos + a
#   complex multiply-add = 15 per direction, is what a form without the symmetries needs.)
#   near field, per (target, source) pair: Laplace 14 (3 differences, |d|^2 in 3 FMA, rsqrt, 1/(4 pi) scale, a
#     complex multiply-add), Helmholtz 24 (the same, k r, sin, cos, two products e^{ikr}/r and a complex
#     multiply-add)
#   normal derivative at the target, per pair: Laplace 21 (the Laplace count with n . d in 3 FMA and 1/r^3 in 3
#     products instead of the scale), Helmholtz 35 (the same, k r, sin, cos, the two factors -(cos + kr sin),
#     kr cos - sin and a complex multiply-add); at the source the same counts (the normal is the source's)
#   gradient at the target, per pair and all three components: Laplace 27 (3 differences, |d|^2 in 3 FMA, rsqrt,
#     1/r^3 in 2 products, then per component d_c / r^3 and its real-by-complex multiply-add: 3 x 5), Helmholtz
#     53 (the same up to 1/r^3, k r in 2 products, sin, cos, the two factors in 2 FMA, then per component d_c / r^3,
#     its two products with the factors and a complex multiply-add: 3 x 11)
#   normal derivative at the source, source transforms: the direction-pair form adds k (s . n) (2 FMA and
#     2 products, 6) and its product with u (2): 24 per 2 directions; the Lagrange anterpolation weights
#     n . grad of the node polynomial (4 products and 2 FMA, 8) before the complex multiply-add (4): 12 per
#     (point, node)
FLOPS_PER_DIRECTION = {"pair": 16.0 / 2, "ring": 22.0 / 4, "pair_dl": 24.0 / 2}
NEAR_FLOPS = {"k_near<false": 14.0, "k_near<true": 24.0, "k_near_dn<false": 21.0, "k_near_dn<true": 35.0,
              "k_near_dl<false": 21.0, "k_near_dl<true": 35.0, "k_near_sym<false": 14.0, "k_near_sym<true": 24.0,
              "k_near_grad<false": 27.0, "k_near_grad<true": 53.0}
# VALU issue slots the implemented near-field loop needs per pair at least (transcendentals co-issue): three FP64
# differences and their conversions to FP32 (6), |d|^2 (3), then Laplace a complex multiply-add (2), Helmholtz
# r = |d|^2 / |d| (1), cos / r and sin / r (2) and a complex multiply-add (4).  The slot utilisation is reported
# separately from the flop fraction.
NEAR_SLOTS = {"k_near<false": 11.0, "k_near<true": 16.0}


def near_model(name, table):
    """The entry of a near-field table for a kernel symbol (its first template argument names the kernel; the
    symmetric derivative pass k_near_sym_d<HELM, BIG, NRM> counts as the ordered kernel it replaces)."""
    if name.startswith("k_near_sym_d<"):
        args = [a.strip() for a in name[len("k_near_sym_d<"):].rstrip(">").split(",")]
        base = {"1": "k_near_dn<", "2": "k_near_dl<", "3": "k_near_grad<"}.get(args[-1])
        return table.get(base + args[0]) if base else None
    for key, v in table.items():
        if name.startswith(key + ",") or name.startswith(key + ">"):
            return v
    return None
# Published MI355X peaks per bound: dense FP32 MFMA 157.3 TFLOP/s, dense FP16 MFMA 2500, FP32 VALU (non-packed,
# FMA = 2) 78.6, HBM3E 8 TB/s.
PEAKS = {"mfma": (157.3, "TFLOP/s"), "mfma16": (2500.0, "TFLOP/s"), "alu": (PEAK_ALU_TFLOPS, "TFLOP/s"),
         "hbm": (8000.0, "GB/s")}

# HBM traffic per launch of the dominant kernel from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of this
# workload (profiles/traffic_apply_helmholtz_sphere_1M.md), scaled by what the counters read for a copy
# kernel of known size (FETCH x 2.0, WRITE x 1.0), mean over the kernel's launches in one product.  Valid only
# for the kernel source it was taken on.
TRAFFIC_SOURCE_HASH = "30968b3507c02672"      # sha256 prefix of paper_1909_05600_amd/csrc/apply.hip
TRAFFIC = {
    "k_pw_forward_rings<2, false>": (35356.281 * 2.0 + 84612.281) * 1024.0,
    "k_grid_phi_s<4>": (202948.312 * 2.0 + 24879.312) * 1024.0,
    "k_grid_phit": (79157.688 * 2.0 + 295680.000) * 1024.0,
    "k_near_sym<true, false>": (201922.000 * 2.0 + 84416.875) * 1024.0,
    "k_pw_transfer_sib": (182038.625 * 2.0 + 56244.031) * 1024.0,
    "k_pw_backward_rings<2, 2, false, 256>": (85142.188 * 2.0 + 24771.500) * 1024.0,
    "k_pw_backward_rings<2, 2, false, 128>": (81293.750 * 2.0 + 25059.125) * 1024.0,
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
    ap.add_argument("--cpu-strides", type=str, default="64,32")
    ap.add_argument("--cpu-validate", type=int, default=0,
                    help="only time the oracle at this N (Helmholtz sphere, ten points per wavelength): the sampled "
                         "estimate and the full product")
    ap.add_argument("--no-batched", action="store_true", help="skip the 256-instance batched workload")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving workload")
    ap.add_argument("--serving-matvecs", type=int, default=50,
                    help="dependent matvecs per session in the serving workload (50, as in a GMRES solve)")
    ap.add_argument("--serving-loads", type=str, default="0.8,1.25",
                    help="offered loads as fractions of the one-at-a-time capacity, e.g. 0.5,0.8,0.95,1.25")
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--mixed-study", action="store_true",
                    help="only run the 10M-point sphere + cube study (FP32 and mixed precision at eps 1e-3, 1e-4)")
    ap.add_argument("--mixed-n", type=int, default=10_000_000)
    ap.add_argument("--bie-study", action="store_true",
                    help="only run the single-layer sphere solve (GMRES with FFM products) at --bie-n nodes")
    ap.add_argument("--bie-n", type=int, default=1 << 20)
    ap.add_argument("--nufft-study", action="store_true",
                    help="bake-off of the grid form's separable sums against an FFT-based type-2 NUFFT")
    ap.add_argument("--aca-study", action="store_true",
                    help="only run the ACA study (full transfer matrices against their ACA factors)")
    ap.add_argument("--deriv-study", action="store_true",
                    help="only time the derivative kernels (normal derivatives, gradient) beside the potential")
    ap.add_argument("--bie-eps", type=float, default=1e-3)
    ap.add_argument("--bie-tol", type=float, default=1e-4)
    ap.add_argument("--mixed-rows", type=int, default=1024)
    return ap.parse_args()


def host_cpu():
    """The host's CPU model and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, usable


def cpu_baseline(w, strides, validate_full=False):
    """The FP64 oracle as it stands, on the host cores.  It builds the full tree, lists and tables, then runs
    the product with only the points whose sorted index is a multiple of s in the per-point loops (source and
    target transforms, near-field targets) for two strides s: every box, table and transfer is kept, so the
    sample has the full product's parallel structure and its point work shrinks by s at every level.  The full product's time is a + b from
    t(s) = a + b / s through the two samples, for the wall time on all threads and for the process's CPU time
    (the core-seconds of the product, the estimate of its time on one core)."""
    import resource
    os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")     # idle threads sleep: CPU time counts work only
    import oracle

    def cpu():
        r = resource.getrusage(resource.RUSAGE_SELF)
        return r.ru_utime + r.ru_stime

    t0, c0 = time.perf_counter(), cpu()
    p = oracle.Plan(w.X, w.X, w.kernel, w.k, w.eps)
    t_plan, c_plan = time.perf_counter() - t0, cpu() - c0
    p.apply(w.wu, stride=1024)       # untimed: starts the thread pool and touches the product's memory
    ts, cs = [], []
    for s in strides:
        t0, c0 = time.perf_counter(), cpu()
        p.apply(w.wu, stride=s)
        ts.append(time.perf_counter() - t0)
        cs.append(cpu() - c0)

    def fit(y):
        (s1, s2), (y1, y2) = strides, y
        b = (y1 - y2) / (1.0 / s1 - 1.0 / s2)
        a = y1 - b / s1
        if b <= 0 or a < 0:          # degenerate fit: all of the sample scales
            a, b = 0.0, y1 * s1
        return a + b

    t_full = t_plan + fit(ts)
    c_full = c_plan + fit(cs)
    model, usable = host_cpu()
    out = {
        "value": w.n / t_full, "unit": "points/s", "cores": oracle.num_threads(), "kind": "oracle",
        "one_core_points_per_s": w.n / c_full, "one_core_s_est": c_full, "all_cores_s_est": t_full,
        "host_cpu": model, "host_cores_usable": usable,
        "sample": "FP64 oracle FFM at N=%d (k=%.3f, eps=%g): full tree, lists and tables (%.1f s), then the product "
                  "with every %d-th and every %d-th point (sorted order) in the per-point loops (%.1f s, %.1f s wall; "
                  "%.1f, %.1f core-s); full product a + b from t(s) = a + b/s: %.0f s on %d threads, %.0f "
                  "core-s (one-core estimate)"
                  % (w.n, w.k, w.eps, t_plan, strides[0], strides[1], ts[0], ts[1], cs[0], cs[1], t_full,
                     oracle.num_threads(), c_full),
    }
    if validate_full:
        t0, c0 = time.perf_counter(), cpu()
        p.apply(w.wu, stride=1)
        out["validation_full_s"] = t_plan + time.perf_counter() - t0
        out["validation_full_core_s"] = c_plan + cpu() - c0
    return out


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
        for prec, adaptive in ((0, False), (1, False), (0, True)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p = ffm.Plan(X, X, 1, w.k, eps, precision=prec, adaptive=adaptive)
            torch.cuda.synchronize()
            t_plan = time.perf_counter() - t0
            v = p.apply(wu)
            t_apply = _sync_time(lambda: p.apply(wu, out=v), reps)
            vv = v.cpu().numpy()[w.rows].astype(np.complex128)
            st = p.stats()

            def rl(a, b):
                return float(np.linalg.norm(a - b) / np.linalg.norm(b))
            r = {"eps": eps, "precision": "mixed" if prec else "fp32", "adaptive_leaves": adaptive,
                 "plan_s": t_plan, "apply_s": t_apply, "early_pairs": [int(x) for x in st["nearly"][:st["leaf"] + 1]],
                 "points_per_s": n / (t_plan + t_apply), "apply_points_per_s": n / t_apply,
                 "err": rl(vv, d), "err_sphere": rl(vv[sph], d[sph]), "err_cube": rl(vv[~sph], d[~sph]),
                 "leaf": st["leaf"], "methods": st["method"][:st["leaf"] + 1],
                 "fp16_levels": [l for l in range(st["leaf"] + 1) if st["prec"][l]],
                 "phase64_levels": [l for l in range(st["leaf"] + 1) if st["phase64"][l]],
                 "plan_mb": st["plan_bytes"] / 1e6, "workspace_mb": st["workspace_bytes"] / 1e6,
                 "dense_rows_s": t_dense}
            out["runs"].append(r)
            print("mixed study eps=%g %s%s: plan %.2fs apply %.3fs err %.2e (sphere %.2e cube %.2e)"
                  % (eps, r["precision"], " adaptive" if adaptive else "", t_plan, t_apply, r["err"], r["err_sphere"],
                     r["err_cube"]),
                  file=sys.stderr, flush=True)
            p.destroy()
            torch.cuda.empty_cache()
    return out


def _es(u, w, beta):
    """Exponential-of-semicircle kernel exp(beta (sqrt(1 - (2u/w)^2) - 1)) on |u| < w/2 (FP64, numpy)."""
    z = 1.0 - (2.0 * u / w) ** 2
    return np.where(np.abs(u) < w / 2, np.exp(beta * (np.sqrt(np.maximum(z, 0.0)) - 1.0)), 0.0)


def nufft_study(n, reps=3):
    """Bake-off of the directions-from-grid step of the grid form (after spreading, which both forms share): the
    separable MFMA sums of this library against the paper's suggested NUFFT route (remark closing Sec. 2.2.3), a
    type-2 NUFFT from the box's grid to the quadrature frequencies k s_q: divide the grid by the frequency
    kernel's inverse transform, zero-pad to (sigma p)^3, 3-D FFT (rocFFT through torch), interpolate the
    spectrum at k s_q with an ES kernel of width wf (a sparse matrix product, hipSPARSE through torch).  Same
    grids, boxes and directions as the 1M-sphere headline plan; times with HIP events, errors against the direct
    sum over the grid in FP64 on 256 directions of one box."""
    import torch
    import ffm_workloads as W
    import paper_1909_05600_amd as ffm
    w = W.helmholtz_sphere(n, seed=2, eps=1e-3)
    X = torch.from_numpy(w.X).cuda()
    wu = torch.from_numpy(w.wu).cuda()
    plan = ffm.Plan(X, X, ffm.FFM_HELMHOLTZ, w.k, w.eps, timing=True)
    ours = {}
    for _ in range(reps):
        plan.apply(wu)
        torch.cuda.synchronize()
        for r in plan.launch_timing():
            ours.setdefault((r["kernel"], r["level"]), []).append(r["ms"])
    st = plan.stats()
    out = {"n": n, "k": w.k, "levels": []}
    dev = torch.device("cuda:0")

    def timed(fn):
        ts = []
        res = None
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            res = fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts)), res

    for l in range(1, st["leaf"] + 1):
        if st["tform"][l] != 3:
            continue
        pg, wg, L = st["grid_nodes"][l], st["grid_width"][l], st["order"][l]
        nb = st["fwd_boxes"][l]
        dl = st["d0"] / 2.0 ** l
        h = dl / (pg - 1 - wg)
        xg, wgl = np.polynomial.legendre.leggauss(L + 1)
        phi = np.pi * np.arange(2 * L) / L
        ct = np.repeat(xg, 2 * L)
        stt = np.sqrt(1.0 - ct ** 2)
        ph = np.tile(phi, L + 1)
        om = w.k * np.stack([stt * np.cos(ph), stt * np.sin(ph), ct], axis=1)     # [nq, 3]
        nq = om.shape[0]
        mine = sum(np.median(v) for (name, lev), v in ours.items()
                   if lev == l and (name.startswith("k_grid_z") and not name.startswith("k_grid_zt")
                                    or name.startswith("k_grid_phi_")))
        lev = {"level": l, "p": pg, "w_spread": wg, "L": L, "nq": nq, "boxes": nb, "kh": w.k * h,
               "grid_form_ms": float(mine), "nufft": []}
        gen = torch.Generator(device=dev).manual_seed(l)
        G = torch.complex(torch.randn((nb, pg, pg, pg), device=dev, generator=gen),
                          torch.randn((nb, pg, pg, pg), device=dev, generator=gen))
        xs = (np.arange(pg) - (pg - 1) / 2) * h
        q0 = np.arange(0, nq, max(1, nq // 256))[:256]
        Eq = [torch.from_numpy(np.exp(-1j * np.outer(om[q0, d], xs))).to(dev) for d in range(3)]
        exact = torch.einsum("abc,qa,qb,qc->q", G[0].to(torch.complex128), Eq[0], Eq[1], Eq[2]).cpu().numpy()
        for sigma, wf in ((2, 5), (2, 6)):
            P = sigma * pg
            Delta = 2 * np.pi / (P * h)
            beta = 2.30 * wf
            tq, wq = np.polynomial.legendre.leggauss(64)
            u = tq * wf / 2
            xsh = (np.arange(pg) - pg // 2) * h                    # grid relative to index pg/2
            phic = (wf / 2) * np.sum(wq[None, :] * _es(u, wf, beta)[None, :] * np.cos(np.outer(xsh, u) * Delta), 1)
            c = torch.from_numpy(1.0 / phic).to(dev, torch.float32)
            t = om / Delta
            m0 = np.floor(t - wf / 2).astype(np.int64) + 1       # [nq, 3]
            offs = np.arange(wf)
            ms = m0[:, :, None] + offs[None, None, :]              # [nq, 3, wf]
            wts = _es(t[:, :, None] - ms, wf, beta)                # [nq, 3, wf]
            mi = ms % P
            flat = (mi[:, 0, :, None, None] * P + mi[:, 1, None, :, None]) * P + mi[:, 2, None, None, :]
            ww = wts[:, 0, :, None, None] * wts[:, 1, None, :, None] * wts[:, 2, None, None, :]
            rows = np.repeat(np.arange(nq), wf ** 3)
            Wsp = torch.sparse_coo_tensor(torch.from_numpy(np.stack([rows, flat.reshape(-1)])),
                                          torch.from_numpy(ww.reshape(-1).astype(np.float32)), (nq, P ** 3),
                                          device=dev).coalesce().to_sparse_csr()
            shift = torch.from_numpy(np.exp(-1j * om.sum(1) * h / 2)).to(dev, torch.complex64)

            def prep():
                pad = torch.zeros((nb, P, P, P), dtype=torch.complex64, device=dev)
                pad[:, :pg, :pg, :pg] = G * c[None, :, None, None] * c[None, None, :, None] * c[None, None, None, :]
                return torch.roll(pad, shifts=(-(pg // 2),) * 3, dims=(1, 2, 3))

            t_prep, pad = timed(prep)
            t_fft, F = timed(lambda: torch.fft.fftn(pad, dim=(1, 2, 3)))
            del pad
            Fm = F.reshape(nb, P ** 3)

            def interp():
                Ft = Fm.transpose(0, 1)
                re = torch.sparse.mm(Wsp, Ft.real.contiguous())
                im = torch.sparse.mm(Wsp, Ft.imag.contiguous())
                return torch.complex(re, im) * shift[:, None]          # [nq, nb]

            t_int, res = timed(interp)
            got = res[q0, 0].cpu().numpy()
            err = float(np.linalg.norm(got - exact) / np.linalg.norm(exact))
            del F, Fm, res, Wsp
            torch.cuda.empty_cache()
            lev["nufft"].append({"sigma": sigma, "wf": wf, "prep_ms": t_prep, "fft_ms": t_fft, "interp_ms": t_int,
                                 "total_ms": t_prep + t_fft + t_int, "err": err,
                                 "grid_bytes": nb * P ** 3 * 8})
            print("nufft study level %d p=%d boxes %d nq %d: grid form %.3f ms; NUFFT sigma %d wf %d: prep %.3f fft %.3f "
                  "interp %.3f ms, err %.2e" % (l, pg, nb, nq, mine, sigma, wf, t_prep, t_fft, t_int, err),
                  file=sys.stderr, flush=True)
        out["levels"].append(lev)
        del G
        torch.cuda.empty_cache()
    plan.destroy()
    return out


def deriv_study(n, reps=5):
    """Apply times of the derivative kernels (Sec. 4.2: the normal derivative at the targets, the double layer,
    the gradient) beside the potential, one plan each over the same N points on the unit sphere with radial unit
    normals and the same input, at the headline wavenumber; each time is the median of reps applies, wall clock
    around a synchronised apply."""
    import torch
    import ffm_workloads as W
    import paper_1909_05600_amd as ffm
    w = W.helmholtz_sphere(n, seed=2, eps=1e-3)
    X = torch.from_numpy(w.X).cuda()
    wu = torch.from_numpy(w.wu).cuda()
    out = {"n": n, "k": w.k, "eps": w.eps, "runs": []}
    for name, kernel, kw in (("potential", ffm.FFM_HELMHOLTZ, {}),
                             ("normal_derivative", ffm.FFM_HELMHOLTZ_DN, {"normals": X}),
                             ("double_layer", ffm.FFM_HELMHOLTZ_DL, {"source_normals": X}),
                             ("gradient", ffm.FFM_HELMHOLTZ_GRAD, {})):
        p = ffm.Plan(X, X, kernel, w.k, w.eps, **kw)
        v = p.apply(wu)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            p.apply(wu, out=v)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        st = p.stats()
        out["runs"].append({"kernel": name, "apply_ms": round(float(np.median(ts)), 3),
                            "transform_form": st["tform"][:st["leaf"] + 1], "plan_mb": round(p.plan_bytes() / 1e6, 1)})
        print("%-18s apply %.2f ms (median of %d)" % (name, float(np.median(ts)), reps), file=sys.stderr, flush=True)
        p.destroy()
    return out


def aca_study(n, reps=5):
    """ACA of the Lagrange transfer matrices (Sec. 2.2.2, eq. ffmACAmatvec) against full matrices: apply and plan
    times, transfer-kernel times and errors against FP64 dense rows, for N points on the sphere: Laplace at
    eps = 1e-4 (six Chebyshev nodes per axis, r = 216) and Helmholtz k = 9 at eps = 1e-3 (Lagrange
    levels with r = 216 and 125); and the 256-instance batched workload in FP32."""
    import torch
    import ffm_workloads as W
    import paper_1909_05600_amd as ffm
    out = {"n": n, "runs": []}
    for kernel, k, eps, seed in ((0, 0.0, 1e-4, 1), (1, 9.0, 1e-3, 2)):
        w = W.helmholtz_sphere(n, seed=seed, k=k, eps=eps, n_rows=256)
        X = torch.from_numpy(w.X).cuda()
        wu = torch.from_numpy(w.wu).cuda()
        d = dense_rows_device(X, wu, kernel, k, w.rows)
        for aca in ("off", "auto"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p = ffm.Plan(X, X, kernel, k, eps, aca=aca, timing=True)
            torch.cuda.synchronize()
            t_plan = time.perf_counter() - t0
            v = p.apply(wu)
            t_apply = _sync_time(lambda: p.apply(wu, out=v), reps)
            lt = p.launch_timing()
            tr = sum(r["ms"] for r in lt if r["kernel"] in ("k_lag_mfma", "k_lag_aca"))
            st = p.stats()
            vv = v.cpu().numpy()[w.rows].astype(np.complex128)
            r = {"kernel": "laplace" if kernel == 0 else "helmholtz", "k": k, "eps": eps, "aca": aca,
                 "plan_s": t_plan, "apply_ms": t_apply * 1e3, "transfer_kernel_ms": tr,
                 "aca_levels": [l for l in range(st["leaf"] + 1) if st["aca"][l]],
                 "mean_rank": [round(st["aca_rank"][l], 1) for l in range(st["leaf"] + 1) if st["method"][l] == 1],
                 "r": [st["order"][l] ** 3 for l in range(st["leaf"] + 1) if st["method"][l] == 1],
                 "err": float(np.linalg.norm(vv - d) / np.linalg.norm(d)), "plan_mb": st["plan_bytes"] / 1e6}
            out["runs"].append(r)
            print("aca study %s eps=%g aca=%s: plan %.2fs apply %.2f ms (transfers %.2f ms) err %.2e"
                  % (r["kernel"], eps, aca, t_plan, r["apply_ms"], tr, r["err"]), file=sys.stderr, flush=True)
            p.destroy()
        del X, wu
        torch.cuda.empty_cache()
    ws = W.batched_instances(256, seed=4)
    Xs = [torch.from_numpy(w.X).cuda() for w in ws]
    wus = [torch.from_numpy(w.wu).cuda() for w in ws]
    n_tot = sum(w.n for w in ws)
    for aca in ("off", "auto"):
        t0 = time.perf_counter()
        plans = [ffm.Plan(X, X, w.kernel, w.k, w.eps, aca=aca) for X, w in zip(Xs, ws)]
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        b = ffm.Batch(plans, graph=True)
        o = b.apply(wus)
        t = _sync_time(lambda: b.apply(wus, outs=o), reps)
        errs = []
        for w, X, u, oo in zip(ws, Xs, wus, o):
            rows = w.rows[:16]
            dd = dense_rows_device(X, u, w.kernel, w.k, rows)
            vv = oo.cpu().numpy()[rows].astype(np.complex128)
            errs.append(float(np.linalg.norm(vv - dd) / np.linalg.norm(dd)))
        nlev = sum(sum(p.stats()["aca"]) for p in plans)
        r = {"workload": "batched 256 instances, FP32 graph", "aca": aca, "points_per_s": n_tot / t,
             "apply_ms": t * 1e3, "plan_s": t_plan, "aca_levels_total": nlev, "err_max": max(errs)}
        out["runs"].append(r)
        print("aca study batched aca=%s: %.3g points/s (%.1f ms), plan %.1fs, %d ACA levels, err max %.2e"
              % (aca, r["points_per_s"], r["apply_ms"], t_plan, nlev, r["err_max"]), file=sys.stderr, flush=True)
        b.destroy()
        for p in plans:
            p.destroy()
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
    """Algorithmic work of one launch of a kernel at a level: (amount, bound, definition), or None for kernels
    without a model here.  mfma / alu amounts are flops (FMA = 2), hbm amounts bytes."""
    L, nq = st["order"][level], st["nq"][level]
    p, w = st["grid_nodes"][level], st["grid_width"][level]
    nbf, nbt = st["fwd_boxes"][level], st["bwd_boxes"][level]
    if name.startswith("k_grid_phi"):
        nb = nbt if name.startswith("k_grid_phit") else nbf
        return (8.0 * nb * (L + 1) * p * p * L, "mfma",
                "8 flops per (box, ring, node a, node b, azimuth): the four real products of the separable "
                "plane sums, FP32 MFMA")
    if name in ("k_grid_z", "k_grid_zt"):
        nb = nbf if name == "k_grid_z" else nbt
        return (8.0 * nb * ((L + 2) // 2) * p ** 3, "mfma",
                "8 flops per (box, ring pair, plane, column): the four real products of the z sums, FP32 MFMA")
    if name.startswith("k_grid_spread"):
        return (4.0 * w ** 3 * st["fwd_points"][level], "alu",
                "4 flops per (point, grid node): the node weight times the complex input, VALU")
    if name.startswith("k_grid_interp"):
        return (4.0 * w ** 3 * st["bwd_points"][level], "alu",
                "4 flops per (point, grid node): a real weight times the complex grid value, VALU")
    if name.startswith("k_pw_forward") or name.startswith("k_pw_backward"):
        pts = st["fwd_points"][level] if "forward" in name else st["bwd_points"][level]
        form = "ring" if "_rings" in name else ("pair_dl" if name.startswith("k_pw_forward_dl") else "pair")
        return (FLOPS_PER_DIRECTION[form] * pts * nq, "alu",
                "flops per (point, direction) of the %s form: %s, VALU + transcendental unit"
                % ("ring-pair" if form == "ring" else "direction-pair",
                   {"ring": "22 per 4 directions", "pair": "16 per 2 directions",
                    "pair_dl": "24 per 2 directions"}[form]))
    if name.startswith("k_near"):
        f = near_model(name, NEAR_FLOPS)
        if f is None:
            return None
        return (f * st["near_pairs"], "alu", "%d flops per (target, source) pair of the near field, VALU" % f)
    if name.startswith("k_pw_transfer"):
        return (8.0 * nq * (nbf + st["nclass"][level] + nbt), "hbm",
                "unique bytes: u~ of every source box, the class tables D and v~ of every target box, 8 per "
                "direction each (the far-pair gathers re-read them from the caches)")
    if name in ("k_lag_mfma", "k_lag_mfma16"):
        r = L ** 3
        return ((8.0 if st.get("_helm") else 4.0) * r * r * st["nfar"][level],
                "mfma16" if name == "k_lag_mfma16" else "mfma",
                "flops of T u~ per far pair, r = r1^3: 8 r^2 (complex T) or 4 r^2 (real T, complex u~); MFMA")
    if name in ("k_lag_anterp", "k_lag_interp"):
        r = L ** 3
        pts = st["fwd_points"][level] if name == "k_lag_anterp" else st["bwd_points"][level]
        return (4.0 * r * pts, "alu", "4 flops per (point, Chebyshev node): a real basis value times complex u, VALU")
    if name == "k_lag_anterp_dl":
        return (12.0 * L ** 3 * st["fwd_points"][level], "alu",
                "12 flops per (point, Chebyshev node): the normal derivative of the node polynomial times complex "
                "u, VALU")
    return None


def roofline(launches, st, steps):
    """Roofline of the dominant kernel (the kernel symbol with the most time per step among those with a work
    model; achieved = its algorithmic work over all its launches / their HIP-event time), and the time-weighted
    fraction of the whole apply, sum over launches of (work / peak of its bound) / the apply's measured time."""
    tot = kernel_totals(launches, steps)
    per = {}
    apply_ms = sum(r["ms"] for step in launches for r in step) / steps
    ideal_ms = 0.0
    for step in launches:
        for r in step:
            m = launch_work(r["kernel"], r["level"], st)
            e = per.setdefault(r["kernel"], {"ms": 0.0, "work": 0.0, "bound": m[1] if m else None,
                                             "definition": m[2] if m else None})
            e["ms"] += r["ms"] / steps
            if m is None:
                continue
            e["work"] += m[0] / steps
            peak, unit = PEAKS[m[1]]
            ideal_ms += m[0] / (peak * (1e12 if unit == "TFLOP/s" else 1e9)) * 1e3 / steps
    per_kernel = {}
    for name, e in per.items():
        if e["bound"] is None or e["ms"] <= 0:
            per_kernel[name] = {"ms": round(e["ms"], 4), "bound": None}
            continue
        peak, unit = PEAKS[e["bound"]]
        rate = e["work"] / (e["ms"] * 1e-3) / (1e12 if unit == "TFLOP/s" else 1e9)
        per_kernel[name] = {"ms": round(e["ms"], 4), "bound": e["bound"], "achieved": round(rate, 3),
                            "unit": unit, "frac": round(rate / peak, 4)}
    per_kernel = dict(sorted(per_kernel.items(), key=lambda kv: -kv[1]["ms"]))
    modelled_ms = sum(v["ms"] for v in per_kernel.values() if v["bound"])
    time_weighted = {"frac": ideal_ms / apply_ms if apply_ms > 0 else 0.0, "apply_ms": apply_ms,
                     "ideal_ms": ideal_ms, "modelled_time_frac": modelled_ms / apply_ms if apply_ms > 0 else 0.0,
                     "definition": "sum over the apply's launches of (algorithmic work / peak of the launch's bound) "
                                   "divided by the apply's measured time (HIP events); launches without a work model "
                                   "count as zero work", "per_kernel": per_kernel}
    for name in tot:
        e = per.get(name)
        if not e or e["bound"] is None or e["ms"] <= 0:
            continue
        peak, unit = PEAKS[e["bound"]]
        rate = e["work"] / (e["ms"] * 1e-3) / (1e12 if unit == "TFLOP/s" else 1e9)
        n = sum(1 for step in launches for r in step if r["kernel"] == name)
        out = {"bound": "alu" if e["bound"] == "alu" else ("hbm" if e["bound"] == "hbm" else "mfma"),
               "kernel": name, "achieved": rate, "peak": peak, "unit": unit, "frac": rate / peak,
               "launches": n // steps, "avg_launch_ms": e["ms"] / max(1, n // steps),
               "work_per_step": e["work"], "work": e["definition"], "time_weighted": time_weighted}
        if e["bound"] == "alu":
            out["peak_packed_fp32"] = PEAK_ALU_PACKED_TFLOPS
            out["frac_of_packed_peak"] = rate / PEAK_ALU_PACKED_TFLOPS
        ns = near_model(name, NEAR_SLOTS)
        if ns is not None:
            out["issue_slot_utilisation"] = ns * st["near_pairs"] / (e["ms"] * 1e-3) / VALU_SLOTS_PER_S
            out["issue_slot_definition"] = ("%d non-transcendental VALU issue slots per pair (the fewest the "
                                            "implemented loop needs) over the 39.3e12 lane-slots/s of the chip"
                                            % ns)
        return name, out
    return "none", {"bound": "alu", "kernel": "none", "achieved": 0.0, "peak": PEAK_ALU_TFLOPS,
                     "unit": "TFLOP/s", "frac": 0.0, "time_weighted": time_weighted}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported"
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

    if args.nufft_study:
        res = {"metric": "plane-wave transforms from the grid: separable MFMA sums against an FFT-based NUFFT",
               "nufft_study": nufft_study(args.n)}
        print(json.dumps(res), flush=True)
        return

    if args.aca_study:
        res = {"metric": "ACA of the Lagrange transfers: apply time and error against full matrices",
               "aca_study": aca_study(args.n)}
        print(json.dumps(res), flush=True)
        return

    if args.deriv_study:
        res = {"metric": "apply time of the derivative kernels beside the potential (N points on the sphere)",
               "deriv_study": deriv_study(args.n)}
        print(json.dumps(res), flush=True)
        return

    if args.cpu_validate:
        wv = W.helmholtz_sphere(args.cpu_validate, seed=2, eps=args.eps)
        strides = tuple(int(x) for x in args.cpu_strides.split(","))
        res = {"metric": "oracle CPU time: sampled estimate against the full product",
               "cpu_validate": cpu_baseline(wv, strides, validate_full=True)}
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
    st["_helm"] = True          # the Helmholtz kernel: complex transfer tables at Lagrange levels
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
        "memory": {"plan_bytes": st["plan_bytes"], "workspace_bytes": st["workspace_bytes"],
                   "tables_bytes": st["plan_bytes"] - st["workspace_bytes"],
                   "plan_bytes_per_point": st["plan_bytes"] / w.n,
                   "tables_bytes_per_point": (st["plan_bytes"] - st["workspace_bytes"]) / w.n,
                   "workspace_bytes_per_point": st["workspace_bytes"] / w.n,
                   "definition": "plan_bytes: all device memory of a plan, its apply workspace included; tables: the "
                                 "rest (trees, lists, operator tables, launch lists)",
                   "paper": "O(N) storage (Sec. 3, Prop. 1); the paper's Table 1 lists about 100 bytes per point "
                            "(Laplace, its own implementation, which keeps nothing between products)"},
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
