#!/usr/bin/env python3
"""Benchmark: one step = one whole registration of the scan-sized workload
(spherical-harmonic surface, template 32,400 points with a cropped cap and
outliers, reference 36,000 points, k = 24 descriptors, 300 iterations of
the shape-weighted gravitational update), on one MI355X.

Prints one JSON line.  `value` is pair interactions per second over the
whole registration (sum over iterations of M*N, divided by the wall time of
the registration including descriptors and the final status read-back).
`roofline` describes the dominant kernel (the all-pairs force kernel),
timed live with HIP events on the stream it is launched on.
`cpu_baseline` times the FP64 C oracle on a bounded sample of the same
force evaluation on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "shape-weighted pair interactions/sec per iteration; ms/registration at fixed RMSE"
PEAK_FP32_TFLOPS = 157.3        # MI355X published FP32 vector peak
LANE_SLOTS_PER_S = 256 * 64 * 2.4e9   # CUs x lanes x clock: one VALU issue slot per lane per clock
# Algorithmic FP32 flops per pair (FMA = 2, transcendentals not counted):
# p = 1: r (3) + similarity exponent (3) + weight (1) + accumulate (6) = 13;
# p = 2: adds q = |r|^2 + eps^2 (6) and the distance factor (1) = 20.
FLOPS_PER_PAIR = {1.0: 13, 2.0: 20}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(pr, E: int, k: int, target_s: float):
    """Time the FP64 C oracle force (one full M x N evaluation, repeated until
    about target_s seconds have passed, or a row sample if one evaluation
    alone is longer) on the host cores."""
    import numpy as np

    from oracle import ref as O

    prm = O.Params(p=1.0, k=k, E=E)
    rng = np.random.default_rng(0)
    aX = rng.uniform(0.0, 0.3, pr.N)     # descriptor values do not change the cost
    aY = rng.uniform(0.0, 0.3, pr.M)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=aX, aY=aY)
    Y = pr.tmpl.astype(np.float64)
    rows = np.arange(min(512, pr.M))
    t0 = time.perf_counter()
    O.forces_c(Y, S, 1000.0, rows=rows)
    t1 = time.perf_counter() - t0
    per_row = t1 / len(rows)
    if per_row * pr.M > target_s:
        rows = np.arange(max(512, int(target_s / per_row)))
        reps = 1
    else:
        rows = None
        reps = max(1, int(round(target_s / (per_row * pr.M))))
    nrows = pr.M if rows is None else len(rows)
    t0 = time.perf_counter()
    for _ in range(reps):
        O.forces_c(Y, S, 1000.0, rows=rows)
    dt = time.perf_counter() - t0
    pairs = reps * nrows * pr.N
    rate = pairs / dt
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": rate, "unit": "pair-interactions/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} FP64 force evaluation(s) (eq. 5) of {nrows} template rows x {pr.N} reference "
                      f"points (p = 1, g = s) by the C oracle in {dt:.1f} s; a {E}-iteration registration "
                      f"would take {pr.M * pr.N * E / rate:.0f} s at this rate (extrapolated)"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--kernel-reps", type=int, default=40)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only: the registration hot path runs on a single "
                                   "MI355X (multi-GPU sharding is a design note, not implemented)",
                          "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    import paper_1902_01061_amd as sg
    from synth import config2

    pr = config2()
    E, k, p = 300, 24, 1.0
    prm = sg.Params(p=p, k=k, E=E)
    M, N = pr.M, pr.N
    log(f"workload: template {M} x reference {N}, k={k}, E={E}, p={p}")
    ctx = sg.Context(0)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    ident = sg.pose_identity()
    pose = ident.clone()

    for w in range(args.warmup):
        pose.copy_(ident)
        ctx.register(tm, rf, prm, pose=pose)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        pose.copy_(ident)
        ctx.register(tm, rf, prm, pose=pose)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {args.steps} registrations: {dt:.3f} s")
    ms_per_step = dt / args.steps * 1e3
    value = M * N * E * args.steps / dt

    # registration quality (pose error against the generating transform, inlier points)
    s_, R_, t_ = sg.pose_to_srt(pose)
    inl = pr.corr >= 0
    Y0 = pr.tmpl[inl].astype(np.float64)
    est = s_ * Y0 @ R_.T + t_
    truth = (Y0 - pr.gt_t) @ pr.gt_R / pr.gt_s
    diam = float(np.linalg.norm(pr.ref.max(0) - pr.ref.min(0)))
    pose_rmse = float(np.sqrt(np.mean(np.sum((est - truth) ** 2, axis=1))))
    nn_rmse = float(ctx.residual(tm, rf, pose).item())

    # dominant kernel: the all-pairs force kernel alone, on the final pose
    a_t, mom_t = ctx.descriptors(tm, k)
    a_r, mom_r = ctx.descriptors(rf, k)
    plan = sg.Plan(ctx, tm, a_t, rf, a_r, mom_t, mom_r, prm)
    for _ in range(3):
        plan.force(pose, t=E - 1, want_wrench=False)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.kernel_reps):
        plan.force(pose, t=E - 1, want_wrench=False)
    e1.record(stream)
    e1.synchronize()
    k_ms = e0.elapsed_time(e1) / args.kernel_reps
    k_pairs = M * N / (k_ms * 1e-3)
    fpp = FLOPS_PER_PAIR[p]
    achieved = fpp * k_pairs / 1e12
    log(f"force kernel: {k_ms:.4f} ms/launch, {k_pairs:.3e} pairs/s, {achieved:.2f} TFLOP/s")
    plan.close()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"scan-sized registration: spherical-harmonic surface, template {M} (25% cap "
                               f"cropped, 15% blob + 5% uniform outliers, 0.8 x 60 deg rotation, noise 0.003) "
                               f"vs reference {N}, k={k} curvature, p={p:g}, g=s, {E} iterations",
                   "M": M, "N": N, "iterations": E, "k": k, "p": p, "g_mode": 0},
        "ms_per_registration": ms_per_step,
        "pose_rmse_over_diameter": pose_rmse / diam,
        "nn_rmse": nn_rmse,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "force_kernel", "ms_per_launch": k_ms, "pairs_per_launch": M * N,
                     "flops_per_pair": fpp, "pairs_per_s": k_pairs},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(pr, E, k, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
