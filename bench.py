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
# Minimal non-transcendental VALU slots of the plane-wave transforms (sin/cos co-issue on the
# transcendental unit at half rate and are not the bound; see profiles/peaks_mi355x.txt):
#   direction-pair form: per (point, antipodal pair)   3 phase + 1 fract + 4 accumulate = 8 slots / 2 directions
#   ring-pair form:      per (point, group of 4 dirs)   2 phase + 1 fract + 8 accumulate = 11 slots / 4 directions
SLOTS_PER_DIRECTION = {1: 8 / 2, 2: 11 / 4}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--eps", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-strides", type=str, default="64,128")
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

    w = W.helmholtz_sphere(args.n, seed=2, eps=args.eps)
    dev = torch.device("cuda:0")
    X = torch.from_numpy(w.X).to(dev)
    wu = torch.from_numpy(w.wu).to(dev)
    out = torch.empty(w.n, dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def step(record):
        t0 = time.perf_counter()
        plan = ffm.Plan(X, X, ffm.FFM_HELMHOLTZ, w.k, w.eps, timing=True)
        t1 = time.perf_counter()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        plan.apply(wu, out=out)
        e1.record(stream)
        e1.synchronize()
        if record is not None:
            record["plan_ms"].append((t1 - t0) * 1e3)
            record["apply_ms"].append(e0.elapsed_time(e1))
            record["phases"].append(plan.timing())
            record["stats"] = plan.stats()
        plan.destroy()

    for _ in range(args.warmup):
        step(None)
    rec = {"plan_ms": [], "apply_ms": [], "phases": [], "stats": None}
    step_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        step(rec)
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    ms_per_step = t_total * 1e3 / args.steps

    st = rec["stats"]
    ph = np.array(rec["phases"])          # [steps][64]
    leaf = st["leaf"]
    # plane-wave transform kernels: forward (slot 1 + 3(l-1)) and backward (slot 3 + 3(l-1))
    fwd_ms = bwd_ms = fwd_slots = bwd_slots = 0.0
    nlaunch = 0
    for l in range(1, leaf + 1):
        if st["method"][l] != 2:
            continue
        per_dir = SLOTS_PER_DIRECTION[st["tform"][l]]
        fwd_ms += ph[:, 1 + 3 * (l - 1)].sum()
        bwd_ms += ph[:, 3 + 3 * (l - 1)].sum()
        fwd_slots += args.steps * st["fwd_points"][l] * st["nq"][l] * per_dir
        bwd_slots += args.steps * st["bwd_points"][l] * st["nq"][l] * per_dir
        nlaunch += args.steps
    dom = "plane-wave forward transform" if fwd_ms >= bwd_ms else "plane-wave backward transform"
    d_ms, d_slots = (fwd_ms, fwd_slots) if fwd_ms >= bwd_ms else (bwd_ms, bwd_slots)
    achieved = 2 * d_slots / (d_ms * 1e-3) / 1e12 if d_ms > 0 else 0.0
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
                   "step": "ffm_plan + ffm_apply + ffm_destroy (the whole product)"},
        "apply_points_per_s": w.n / (np.mean(rec["apply_ms"]) * 1e-3),
        "apply_ms": float(np.mean(rec["apply_ms"])),
        "plan_ms": float(np.mean(rec["plan_ms"])),
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99))},
        "phases_ms": phases,
        "roofline": {
            "bound": "alu", "kernel": dom, "achieved": achieved, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_ALU_TFLOPS, "traffic": None,
            "launches": nlaunch, "avg_launch_ms": d_ms / max(nlaunch, 1),
            "work": "non-transcendental VALU issue slots x 2 (FMA-equivalent flops) of the implemented form: "
                    "11 per (point, 4 directions) in ring-pair levels, 8 per (point, 2 directions) otherwise; "
                    "peak = 256 CU x 64 lanes x 2.4 GHz x 2",
        },
        "levels": {"leaf": leaf, "nq": [int(x) for x in st["nq"][:leaf + 1]],
                   "transform_form": [int(x) for x in st["tform"][:leaf + 1]],
                   "nfar": [int(x) for x in st["nfar"][:leaf + 1]], "near_pairs": st["near_pairs"],
                   "transform_terms": st["transform_terms"]},
    }
    if not args.no_cpu_baseline:
        strides = tuple(int(s) for s in args.cpu_strides.split(","))
        res["cpu_baseline"] = cpu_baseline(w, strides)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
