#!/usr/bin/env python3
"""Benchmark: one step = one whole registration of the largest single-GPU
workload, the depth-frame scene (reference 307,200 points: a 640 x 480
frame of a room with 20 boxes; template 250,000 points of the same room
after one box is removed and two are added, seen from a camera turned
30 degrees; k = 16 curvature, g = a a s (eq. 10), p = 1, 100 iterations of
the shape-weighted gravitational update), on one MI355X.

Prints one JSON line.  `value` is pair interactions per second over the
whole registration (sum over iterations of M*N, divided by the wall time of
the registration including descriptors and the final status read-back).
`roofline` describes the dominant kernel (the all-pairs force kernel),
timed live with HIP events on the stream it is launched on; `roofline_rform`
is the same kernel with the distance law of p = 2 (eq. 11: one log2 and one
exp2 per pair) at the same size.  `cpu_baseline` times the FP64 C oracle on
a bounded sample of rows of the same force evaluation on the host cores.
The scan-sized pair (32,400 x 36,000, 300 iterations) and the other
workloads are extra legs.  Every pose error is printed beside the error of
the identity pose and of the scale-only update (the pose after a first
iteration with no force) for the same pair.
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
# Without packed FP32 (every HIP unit of the library is compiled without it) a lane
# retires one FP32 FMA per clock: 256 CU x 64 lanes x 2 flops x 2.4 GHz.
PEAK_FP32_UNPACKED_TFLOPS = 78.6
LANE_SLOTS_PER_S = 256 * 64 * 2.4e9   # CUs x lanes x clock: one VALU issue slot per lane per clock
# Algorithmic FP32 flops per pair (FMA = 2, transcendentals not counted):
# p = 1: r (3) + similarity exponent (3) + weight (1) + accumulate (6) = 13;
# p = 2: adds q = |r|^2 + eps^2 (6) and the distance factor (1) = 20.
FLOPS_PER_PAIR = {1.0: 13, 2.0: 20}
TILES = os.path.join(ROOT, "paper_1902_01061_amd", "tiles_gfx950.json")
# Counter summaries (FETCH_SIZE, WRITE_SIZE) of the force kernel, by (M, N, p).
COUNTERS = {(250000, 307200, 1.0): os.path.join(ROOT, "profiles", "force_kernel_scene_250000x307200_counters.json"),
            (250000, 307200, 2.0): os.path.join(ROOT, "profiles",
                                                "force_kernel_rform_scene_250000x307200_counters.json")}
FORCE_SOURCES = ["paper_1902_01061_amd/csrc/force.hip", "paper_1902_01061_amd/csrc/common.h"]


def _log2_bucket(n: int) -> int:
    return n.bit_length() - 1


def _launch_of(path, M, N, p):
    """The launch shape the library will use for (M, N, p) from a tile table."""
    pm = 1 if p == 1.0 else (3 if p == 3.0 else 0)
    with open(path) as f:
        tab = json.load(f)
    for e in tab["entries"]:
        if (e["m_bucket"], e["n_bucket"], e["p_mode"]) == (_log2_bucket(M), _log2_bucket(N), pm):
            return {"R": e["R"], "blocks_per_cu": e["blocks_per_cu"], "variant": e["variant"]}
    return None


def _sources_digest():
    import hashlib

    h = hashlib.sha256()
    for rel in FORCE_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _traffic(launch, M, N, p):
    """HBM bytes per launch of the force kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by the copy calibration), or
    None when there is none for this workload, or the kernel source or its
    launch shape changed since."""
    path = COUNTERS.get((M, N, p))
    if launch is None or path is None or not os.path.exists(path):
        return None
    with open(path) as f:
        c = json.load(f)
    if c.get("sources_sha256") != _sources_digest() or c.get("launch") != launch:
        return None
    return c["traffic_bytes_per_launch"]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(pr, E: int, k: int, target_s: float, g_mode: int = 0):
    """Time the FP64 C oracle force on the host cores: on all host threads
    (one full M x N evaluation, repeated until about target_s seconds have
    passed, or a row sample if one evaluation alone is longer), then on one
    thread over a row sample of about target_s / 3 seconds."""
    import numpy as np

    from oracle import ref as O

    prm = O.Params(p=1.0, g_mode=g_mode, k=k, E=E)
    rng = np.random.default_rng(0)
    aX = rng.uniform(0.0, 0.3, pr.N)     # descriptor values do not change the cost
    aY = rng.uniform(0.0, 0.3, pr.M)
    S = O.make_setup(pr.ref, pr.tmpl, prm, aX=aX, aY=aY)
    Y = pr.tmpl.astype(np.float64)

    def timed_rate(budget_s):
        rows = np.arange(min(512, pr.M))
        t0 = time.perf_counter()
        O.forces_c(Y, S, 1000.0, rows=rows)
        per_row = (time.perf_counter() - t0) / len(rows)
        if per_row * pr.M > budget_s:
            rows = np.arange(max(64, min(pr.M, int(budget_s / per_row))))
            reps = 1
        else:
            rows = None
            reps = max(1, int(round(budget_s / (per_row * pr.M))))
        nrows = pr.M if rows is None else len(rows)
        t0 = time.perf_counter()
        for _ in range(reps):
            O.forces_c(Y, S, 1000.0, rows=rows)
        dt = time.perf_counter() - t0
        return reps * nrows * pr.N / dt, reps, nrows, dt

    all_threads = O.c_threads()
    rate, reps, nrows, dt = timed_rate(target_s)
    O.c_threads(1)
    rate1, _, nrows1, dt1 = timed_rate(target_s / 3)
    O.c_threads(all_threads)
    return {"value": rate, "unit": "pair-interactions/s", "cores": all_threads, "kind": "oracle",
            "sample": f"{reps} FP64 force evaluation(s) (eq. 5) of {nrows} template rows x {pr.N} reference "
                      f"points (p = 1, g = {'a a s' if g_mode == 1 else 's'}) by the C oracle on {all_threads} "
                      f"threads in {dt:.1f} s; a "
                      f"{E}-iteration registration would take {pr.M * pr.N * E / rate:.0f} s at this rate "
                      f"(extrapolated)",
            "single_thread": {"value": rate1, "unit": "pair-interactions/s", "cores": 1,
                              "sample": f"{nrows1} template rows x {pr.N} reference points in {dt1:.1f} s"}}


def _pose_err(sg, pose, pr):
    """Pose RMSE over inlier template points against the generating transform,
    divided by the reference bounding-box diagonal."""
    import numpy as np

    s_, R_, t_ = sg.pose_to_srt(pose)
    inl = pr.corr >= 0
    Y0 = pr.tmpl[inl] if inl.any() else pr.tmpl
    Y0 = Y0.astype(np.float64)
    est = s_ * Y0 @ R_.T + t_
    truth = (Y0 - pr.gt_t) @ pr.gt_R / pr.gt_s
    diam = float(np.linalg.norm(pr.ref.max(0) - pr.ref.min(0)))
    return float(np.sqrt(np.mean(np.sum((est - truth) ** 2, axis=1)))) / diam


def _pose_err_srt(s_, R_, t_, pr):
    """_pose_err for a pose given as (s, R, t) on the host."""
    import numpy as np

    inl = pr.corr >= 0
    Y0 = (pr.tmpl[inl] if inl.any() else pr.tmpl).astype(np.float64)
    est = s_ * Y0 @ np.asarray(R_).T + t_
    truth = (Y0 - pr.gt_t) @ pr.gt_R / pr.gt_s
    diam = float(np.linalg.norm(pr.ref.max(0) - pr.ref.min(0)))
    return float(np.sqrt(np.mean(np.sum((est - truth) ** 2, axis=1)))) / diam


def _reference_errors(pr):
    """Pose errors that frame a registration's: the identity pose, and the
    scale-only update (what the first iteration does when every force is
    zero: the template scaled about its centroid by sqrt(lambda_max(Sigma_X)
    / lambda_max(Sigma_Y)), eq. 8)."""
    import numpy as np

    def lam(P):
        Q = P.astype(np.float64)
        Q = Q - Q.mean(0)
        return float(np.linalg.eigvalsh(Q.T @ Q / len(Q))[-1])

    c = float(np.sqrt(lam(pr.ref) / lam(pr.tmpl)))
    yb = pr.tmpl.astype(np.float64).mean(0)
    return {"identity_pose_rmse_over_diameter": _pose_err_srt(1.0, np.eye(3), np.zeros(3), pr),
            "scale_only_pose_rmse_over_diameter": _pose_err_srt(c, np.eye(3), yb - c * yb, pr)}


def _timed(fn, reps=1):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, out


def extra_batch(sg, ctx):
    """256 uneven registrations in one batched call, and a 32-start sweep."""
    import numpy as np

    from synth import config4, config4_multistart

    pairs = config4()
    E = 100
    prm = sg.Params(p=1.0, k=16, E=E)
    tms = [sg.Cloud(p.tmpl) for p in pairs]
    rfs = [sg.Cloud(p.ref) for p in pairs]
    ctx.register_batch(tms, rfs, prm)             # warm-up (graph capture)
    dt, (poses, energy, _) = _timed(lambda: ctx.register_batch(tms, rfs, prm))
    pairs_total = sum(p.M * p.N for p in pairs) * E
    errs = [_pose_err(sg, poses[r], pr) for r, pr in enumerate(pairs)]
    ms_pr, R0 = config4_multistart()
    tm, rf = sg.Cloud(ms_pr.tmpl), sg.Cloud(ms_pr.ref)
    ctx.multistart(tm, rf, prm, R0)
    dtm, (mposes, menergy, best) = _timed(lambda: ctx.multistart(tm, rf, prm, R0))
    start_err = [_pose_err(sg, mposes[s], ms_pr) for s in range(len(R0))]
    # the same batch and sweep with the p = 1 pair sums formed once (flags bit 3)
    prm_i = sg.Params(p=1.0, k=16, E=E, flags=8)
    ctx.register_batch(tms, rfs, prm_i)
    dti, (poses_i, _, _) = _timed(lambda: ctx.register_batch(tms, rfs, prm_i))
    ctx.multistart(tm, rf, prm_i, R0)
    dtmi, (mposes_i, _, best_i) = _timed(lambda: ctx.multistart(tm, rf, prm_i, R0))
    dp = max(abs(_pose_err(sg, poses_i[r], pr) - errs[r]) for r, pr in enumerate(pairs))
    return {"registrations": len(pairs), "points_range": [min(p.N for p in pairs), max(p.N for p in pairs)],
            "iterations": E, "ms_per_batch": dt * 1e3, "pairs_per_s": pairs_total / dt,
            "pose_rmse_over_diameter_median": float(np.median(errs)),
            "multistart": {"starts": len(R0), "M": ms_pr.M, "N": ms_pr.N, "ms": dtm * 1e3,
                           "pairs_per_s": len(R0) * ms_pr.M * ms_pr.N * E / dtm, "best_start": best,
                           "best_pose_rmse_over_diameter": start_err[best],
                           "min_pose_rmse_over_diameter": float(min(start_err))},
            "pose_independent_sums": {"ms_per_batch": dti * 1e3, "speedup": dt / dti, "multistart_ms": dtmi * 1e3,
                                      "multistart_speedup": dtm / dtmi, "multistart_best_start": best_i,
                                      "max_pose_error_change_over_diameter": dp}}


def extra_adjoint(sg, ctx):
    """Forward + adjoint of the force field at 8192 x 8192 (p = 2, eps = 0.05 L)."""
    import numpy as np
    import torch

    from synth import config3

    pr = config3()
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    a_t, _ = ctx.descriptors(tm, 16)
    a_r, mom_r = ctx.descriptors(rf, 16)
    L = float(np.sqrt(mom_r[9].item()))
    sigma = float(a_r.double().std(unbiased=False).item())
    prm = sg.Params(p=2.0, k=16, sigma=sigma, eps=0.05 * L)
    G = 5000.0
    gf = torch.randn((pr.M, 3), device="cuda")
    fwd = lambda: ctx.force_fwd(tm, a_t, rf, a_r, mom_r, prm, G)
    f, _ = fwd()
    bwd = lambda: ctx.force_bwd(tm, a_t, rf, a_r, mom_r, prm, G, f, gf, None)
    bwd()
    tf, _ = _timed(fwd, 20)
    tb, (gy, gm, gse) = _timed(bwd, 20)
    out = {"M": pr.M, "N": pr.N, "p": 2, "fwd_ms": tf * 1e3, "bwd_ms": tb * 1e3,
           "fwd_pairs_per_s": pr.M * pr.N / tf, "bwd_pairs_per_s": pr.M * pr.N / tb,
           "grads_finite": bool(torch.isfinite(gy).all().item() and torch.isfinite(gse).all().item())}

    # 50 unrolled iterations with pose checkpoints every 10, differentiated
    # w.r.t. (sigma, eps, initial pose); the loss is the squared pose error
    # against the generating transform on the inlier template points.
    E, K = 50, 10
    a_t, mom_t = ctx.descriptors(tm, 16)
    prm_u = sg.Params(p=2.0, k=16, sigma=sigma, eps=0.05 * L, E=E)
    inl = pr.corr >= 0
    Yi = torch.as_tensor(pr.tmpl[inl], dtype=torch.float64, device="cuda")
    Zi = torch.as_tensor((pr.tmpl[inl].astype(np.float64) - pr.gt_t) @ pr.gt_R / pr.gt_s, dtype=torch.float64,
                         device="cuda")

    def loss_of(pose):
        est = pose[0] * Yi @ pose[1:10].view(3, 3).T + pose[10:13]
        return ((est - Zi) ** 2).sum(dim=1).mean()

    def run(log_sigma):
        ls = torch.tensor(log_sigma, dtype=torch.float64, requires_grad=True)
        eps = torch.tensor(0.05 * L, dtype=torch.float64, requires_grad=True)
        p0 = sg.pose_identity().requires_grad_(True)
        pose = sg.UnrolledRegistration.apply(ls.exp(), eps, p0, ctx, tm, a_t, rf, a_r, mom_t, mom_r, prm_u, K)
        lo = loss_of(pose)
        lo.backward()
        return float(lo.item()), float(ls.grad.item()), float(eps.grad.item())

    run(np.log(sigma))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lo0, g0, ge0 = run(np.log(sigma))
    torch.cuda.synchronize()
    t_fb = time.perf_counter() - t0
    pose_f, _ = ctx.unrolled_fwd(tm, a_t, rf, a_r, mom_t, mom_r, prm_u, K)
    t_f, _ = _timed(lambda: ctx.unrolled_fwd(tm, a_t, rf, a_r, mom_t, mom_r, prm_u, K), 3)
    # bandwidth tuning: a few gradient steps on log sigma, the first one of size 0.2
    traj = [(sigma, lo0)]
    ls, g = float(np.log(sigma)), g0
    eta = 0.2 / max(abs(g), 1e-300)
    for _ in range(4):
        ls -= eta * g
        lo, g, _ = run(ls)
        traj.append((float(np.exp(ls)), lo))
    out["unrolled"] = {"iterations": E, "checkpoint_every": K, "fwd_ms": t_f * 1e3,
                       "fwd_plus_bwd_ms": t_fb * 1e3, "loss": lo0, "dloss_dlog_sigma": g0, "dloss_deps": ge0,
                       "sigma_tuning": [{"sigma": a, "loss": b} for a, b in traj]}
    return out


def extra_force_law(sg, ctx, E: int, k: int):
    """The method's force law (p = 1, g = s, eq. 5 with eqs. 3, 11) against
    the gravitational law of eq. (1) (p = -2, softening eps = 0.05 L, g = 1:
    no shape term), both with the G schedule of eq. 12, on the workload pair
    and on the small pair: time and pose error after E iterations."""
    import numpy as np

    from synth import config1, config2

    out = {}
    for name, pr in (("small", config1()), ("workload", config2())):
        tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
        L = float(np.sqrt(np.linalg.eigvalsh(np.cov(pr.ref.astype(np.float64).T, bias=True))[-1]))
        row = {"M": pr.M, "N": pr.N, "iterations": E}
        for law, prm in (("shape_p1", sg.Params(p=1.0, k=k, E=E)),
                         ("gravitational_p-2", sg.Params(p=-2.0, g_mode=2, eps=0.05 * L, k=k, E=E))):
            pose = sg.pose_identity()
            ctx.register(tm, rf, prm, pose=pose)
            dt, _ = _timed(lambda: (pose.copy_(sg.pose_identity()), ctx.register(tm, rf, prm, pose=pose)))
            row[law] = {"ms_per_registration": dt * 1e3, "pose_rmse_over_diameter": _pose_err(sg, pose, pr),
                        "nn_rmse": float(ctx.residual(tm, rf, pose).item())}
        out[name] = row
    return out


def extra_pyramid(sg, ctx, E: int, k: int):
    """Radius-neighbourhood curvature (Sec. IV, radius sqrt(lambda_max)) on
    the workload reference, timed alone, and the pyramidal schedule (radius
    and sigma halved twice over the E iterations) against the kNN
    registration on the workload pair."""
    import numpy as np
    import torch

    from synth import config2

    pr = config2()
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    _, mom = ctx.descriptors(rf, k)
    r2 = float(np.float32(mom[9].item()))
    ctx.descriptors_radius(rf, r2)
    reps = 5
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        a, cnt = ctx.descriptors_radius(rf, r2)
    e1.record()
    torch.cuda.synchronize()
    r_ms = e0.elapsed_time(e1) / reps
    third = E // 3
    levels = [sg.Level(1.0, 1.0, third), sg.Level(0.5, 0.5, third), sg.Level(0.25, 0.25, E - 2 * third)]
    prm = sg.Params(p=1.0, k=k, E=E)
    out = {"radius_descriptors": {"N": pr.N, "ms": r_ms, "pair_tests_per_s": pr.N * pr.N / (r_ms * 1e-3),
                                  "members_mean": float(cnt.float().mean().item())},
           "levels": [[v.radius_scale, v.sigma_scale, v.iters] for v in levels]}
    for name, fn in (("knn", lambda p: ctx.register(tm, rf, prm, pose=p)),
                     ("pyramid", lambda p: ctx.register_pyramid(tm, rf, prm, levels, pose=p))):
        pose = sg.pose_identity()
        fn(pose)
        dt, _ = _timed(lambda: (pose.copy_(sg.pose_identity()), fn(pose)))
        out[name] = {"ms_per_registration": dt * 1e3, "pose_rmse_over_diameter": _pose_err(sg, pose, pr),
                     "nn_rmse": float(ctx.residual(tm, rf, pose).item())}
    return out


def extra_vector(sg, ctx, E: int, k: int, D: int = 16):
    """Vector shape descriptors on the workload pair: the soft histograms of
    normals (D bins) of both clouds, then the registration whose pair
    exponents are a contraction on the matrix cores, in its two forms: split
    f16 (heads and tails as one contraction of length 3 (D + 2), two 16x16x32
    f16 instructions per 16 x 16 block for D = 16; peak 2.5 PFLOP/s) and FP32 products (K = 4 ceil((D + 2) / 4); peak 157.3
    TFLOP/s).  Matrix rate = matrix flops of all pairs of all iterations /
    registration time: a lower bound, since the time includes set-up and
    updates."""
    import torch

    from synth import config2

    pr = config2()
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    ctx.descriptors_hn(rf, k, D)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hX = ctx.descriptors_hn(rf, k, D)
    hY = ctx.descriptors_hn(tm, k, D)
    torch.cuda.synchronize()
    d_ms = (time.perf_counter() - t0) * 1e3
    out = {"D": D, "M": pr.M, "N": pr.N, "iterations": E, "descriptors_ms_both_clouds": d_ms}
    pairs = pr.M * pr.N * E
    for form, flags, fpp, peak in (("split_f16", 0, 2 * 32 * ((3 * (D + 2) + 31) // 32), 2500.0),
                                   ("fp32", 4, 2 * 4 * ((D + 2 + 3) // 4), 157.3)):
        prm = sg.Params(p=1.0, k=k, E=E, flags=flags)
        pose = sg.pose_identity()
        ctx.register_vec(tm, hY, rf, hX, prm, pose=pose)
        dt, _ = _timed(lambda: (pose.copy_(sg.pose_identity()), ctx.register_vec(tm, hY, rf, hX, prm, pose=pose)))
        out[form] = {"ms_per_registration": dt * 1e3, "pairs_per_s": pairs / dt, "matrix_flops_per_pair": fpp,
                     "matrix_tflops_lower_bound": fpp * pairs / dt / 1e12,
                     "matrix_peak_tflops": peak, "frac_lower_bound": fpp * pairs / dt / 1e12 / peak,
                     "pose_rmse_over_diameter": _pose_err(sg, pose, pr),
                     "nn_rmse": float(ctx.residual(tm, rf, pose).item())}
    # local polynomial descriptors (D = 3: fitted Hessian eigenvalues, residual)
    ctx.descriptors_poly(rf, k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pX = ctx.descriptors_poly(rf, k)
    pY = ctx.descriptors_poly(tm, k)
    torch.cuda.synchronize()
    dp_ms = (time.perf_counter() - t0) * 1e3
    prm = sg.Params(p=1.0, k=k, E=E)
    pose = sg.pose_identity()
    ctx.register_vec(tm, pY, rf, pX, prm, pose=pose)
    dt, _ = _timed(lambda: (pose.copy_(sg.pose_identity()), ctx.register_vec(tm, pY, rf, pX, prm, pose=pose)))
    out["poly_descriptors"] = {"D": 3, "descriptors_ms_both_clouds": dp_ms, "ms_per_registration": dt * 1e3,
                               "pose_rmse_over_diameter": _pose_err(sg, pose, pr)}
    # split f16 with the pair sums formed by one pass of the kernel (flags bit 3)
    prm = sg.Params(p=1.0, k=k, E=E, flags=8)
    pose = sg.pose_identity()
    ctx.register_vec(tm, hY, rf, hX, prm, pose=pose)
    dt, _ = _timed(lambda: (pose.copy_(sg.pose_identity()), ctx.register_vec(tm, hY, rf, hX, prm, pose=pose)))
    out["split_f16_pose_independent_sums"] = {"ms_per_registration": dt * 1e3,
                                              "speedup": out["split_f16"]["ms_per_registration"] / (dt * 1e3),
                                              "pose_rmse_over_diameter": _pose_err(sg, pose, pr)}
    return out


def extra_scene(sg, ctx, pr, fp32_dt, fp32_pose):
    """The headline scene's other forms: the mixed-precision registration,
    its pose difference from the FP32 one per iteration, the pose-independent
    pair sums, and change detection (their force parity with the oracle along
    the FP32 trajectory is a test: tests/test_gpu_edges.py)."""
    import numpy as np
    import torch

    E = 100
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    out = {"M": pr.M, "N": pr.N, "iterations": E, "g_mode": 1}
    res = {"fp32": (fp32_dt, fp32_pose, None)}
    prm_m = sg.Params(p=1.0, g_mode=1, k=16, E=E, flags=2)
    ctx.register(tm, rf, prm_m)
    dt, (pose, _) = _timed(lambda: ctx.register(tm, rf, prm_m))
    res["mixed"] = (dt, pose, None)
    out["mixed"] = {"ms_per_registration": dt * 1e3, "pairs_per_s": pr.M * pr.N * E / dt,
                    "pose_rmse_over_diameter": _pose_err(sg, pose, pr)}
    for name, flags in (("fp32", 0), ("mixed", 2)):
        _, st = ctx.register(tm, rf, sg.Params(p=1.0, g_mode=1, k=16, E=E, flags=flags), stats=True)  # untimed
        res[name] = (res[name][0], res[name][1], st.cpu().numpy())
    out["mixed_speedup"] = res["fp32"][0] / res["mixed"][0]
    # per-iteration pose difference, mixed vs FP32, as RMSE of transformed template points / diameter
    diam = float(np.linalg.norm(pr.ref.max(0) - pr.ref.min(0)))
    sub = pr.tmpl[:: max(1, pr.M // 5000)].astype(np.float64)
    def apply(row):
        s_, R_, t_ = row[14], row[15:24].reshape(3, 3), row[24:27]
        return s_ * sub @ R_.T + t_
    # the same registration with the pair sums formed once (flags bit 3)
    prm_i = sg.Params(p=1.0, g_mode=1, k=16, E=E, flags=8)
    ctx.register(tm, rf, prm_i)
    dti, (pose_i, _) = _timed(lambda: ctx.register(tm, rf, prm_i))
    s0, R0, t0 = sg.pose_to_srt(res["fp32"][1])
    si, Ri, ti = sg.pose_to_srt(pose_i)
    dpi = float(np.sqrt(np.mean(np.sum(((si * sub @ Ri.T + ti) - (s0 * sub @ R0.T + t0)) ** 2, 1)))) / diam
    out["pose_independent_sums"] = {"ms_per_registration": dti * 1e3, "speedup_vs_fp32": res["fp32"][0] / dti,
                                    "pose_difference_vs_fp32_over_diameter": dpi}
    diffs = [float(np.sqrt(np.mean(np.sum((apply(res["mixed"][2][t]) - apply(res["fp32"][2][t])) ** 2, 1)))) / diam
             for t in range(E)]
    out["mixed_vs_fp32_pose_diff_per_iter"] = {"t0..4": diffs[:5], "t10": diffs[10], "t50": diffs[50],
                                                 "t99": diffs[99]}
    a_t, _ = ctx.descriptors(tm, 16)
    a_r, _ = ctx.descriptors(rf, 16)

    # Change detection: template points with nothing within tau of their
    # registered position (added objects), and the reverse under the inverse
    # pose (removed objects), at the generating transform and at the FP32
    # registration's pose, scored against the scene's own change labels.
    tau, s_min = 0.05, 0.0
    sigma = float(a_r.double().std(unbiased=False).item())
    R_inv = pr.gt_R.T
    gt = torch.tensor(np.concatenate([[1.0 / pr.gt_s], R_inv.reshape(-1), -(R_inv @ pr.gt_t) / pr.gt_s]),
                      dtype=torch.float64, device="cuda")
    # template points that fall inside the reference camera's image (no
    # occlusion test): outside it the reference has no data at all
    Xc = (pr.tmpl.astype(np.float64) - pr.gt_t) @ pr.gt_R / pr.gt_s
    with np.errstate(divide="ignore", invalid="ignore"):
        in_view = (Xc[:, 2] > 0) & (np.abs(Xc[:, 0] / Xc[:, 2]) <= 319.5 / 525) & \
                  (np.abs(Xc[:, 1] / Xc[:, 2]) <= 239.5 / 525)
    cd = {"tau": tau, "template_points_in_reference_view": int(in_view.sum())}
    for name, pose in (("generating_transform", gt), ("fp32_registration", res["fp32"][1])):
        dt_f, (f, _, _) = _timed(lambda: ctx.change_detect(tm, a_t, rf, a_r, pose, tau, sigma, s_min), 3)
        inv = sg.pose_inverse(pose)
        dt_r, (g, _, _) = _timed(lambda: ctx.change_detect(rf, a_r, tm, a_t, inv, tau, sigma, s_min), 3)
        hit = (f.cpu().numpy() & 1) > 0
        ghit = (g.cpu().numpy() & 1) > 0
        cd[name] = {"ms_template_to_reference": dt_f * 1e3, "ms_reference_to_template": dt_r * 1e3,
                    "added_recall": float(hit[pr.changed].mean()),
                    "flag_rate_unchanged_in_reference_view": float(hit[~pr.changed & in_view].mean()),
                    "flag_rate_unchanged_all": float(hit[~pr.changed].mean()),
                    "removed_recall": float(ghit[pr.ref_changed].mean()),
                    "reverse_flag_rate_unchanged": float(ghit[~pr.ref_changed].mean())}
    out["change_detection"] = cd
    return out


def extra_scan(sg, ctx, steps: int, kernel_reps: int):
    """The scan-sized pair (32,400 x 36,000, k = 24, g = s, 300 iterations):
    registration time and pose error beside the identity and scale-only
    errors, the number of template rows whose force is not negligible at the
    first iterate (with the default sigma, the smooth reference's curvatures
    lie far below the noisy template's, and most rows' weights underflow),
    the force kernel alone, and the mixed-precision and pose-independent
    forms."""
    import numpy as np
    import torch

    from synth import config2

    pr = config2()
    E, k = 300, 24
    prm = sg.Params(p=1.0, k=k, E=E)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    ident = sg.pose_identity()
    out = {"M": pr.M, "N": pr.N, "iterations": E, "k": k}
    forms = {}
    for name, flags in (("fp32", 0), ("mixed", 2), ("pose_independent_sums", 8)):
        pp = sg.Params(p=1.0, k=k, E=E, flags=flags)
        pose = ident.clone()
        ctx.register(tm, rf, pp, pose=pose)
        dt, _ = _timed(lambda: (pose.copy_(ident), ctx.register(tm, rf, pp, pose=pose)), steps)
        forms[name] = (dt, pose)
        out[name] = {"ms_per_registration": dt * 1e3, "pairs_per_s": pr.M * pr.N * E / dt,
                     "pose_rmse_over_diameter": _pose_err(sg, pose, pr)}
    out["fp32"]["nn_rmse"] = float(ctx.residual(tm, rf, forms["fp32"][1]).item())
    out["mixed"]["speedup_vs_fp32"] = forms["fp32"][0] / forms["mixed"][0]
    out["pose_independent_sums"]["speedup_vs_all_pairs"] = forms["fp32"][0] / forms["pose_independent_sums"][0]
    out.update(_reference_errors(pr))
    a_t, mom_t = ctx.descriptors(tm, k)
    a_r, mom_r = ctx.descriptors(rf, k)
    plan = sg.Plan(ctx, tm, a_t, rf, a_r, mom_t, mom_r, prm)
    _, f = plan.force(ident, t=0, want_wrench=False, want_f=True)
    fn = torch.linalg.vector_norm(f.double(), dim=1)
    out["rows_with_force_at_t0"] = int((fn > 1e-6 * fn.max()).sum().item())
    for _ in range(3):
        plan.force(forms["fp32"][1], t=E - 1, want_wrench=False)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(kernel_reps):
        plan.force(forms["fp32"][1], t=E - 1, want_wrench=False)
    e1.record(stream)
    e1.synchronize()
    k_ms = e0.elapsed_time(e1) / kernel_reps
    plan.close()
    out["force_kernel"] = {"ms_per_launch": k_ms, "pairs_per_s": pr.M * pr.N / (k_ms * 1e-3),
                           "tflops_13_per_pair": 13 * pr.M * pr.N / (k_ms * 1e-3) / 1e12}
    # the r-form of the same kernel on this pair: the p = 2 law (20 flops per
    # pair) and eq. 1's gravitational law (p = -2, eps = 0.05 L, g = 1)
    L = float(np.sqrt(mom_r[9].item()))
    for name, pp in (("force_kernel_p2", sg.Params(p=2.0, k=k, E=E)),
                     ("force_kernel_gravitational_p-2", sg.Params(p=-2.0, g_mode=2, eps=0.05 * L, k=k, E=E))):
        pl = sg.Plan(ctx, tm, a_t, rf, a_r, mom_t, mom_r, pp)
        ms = _kernel_ms(pl, forms["fp32"][1], E - 1, kernel_reps)
        pl.close()
        out[name] = {"ms_per_launch": ms, "pairs_per_s": pr.M * pr.N / (ms * 1e-3)}
    return out


def _kernel_ms(plan, pose, t, reps):
    """Average duration of the force kernel alone: HIP events around `reps`
    back-to-back launches on the stream the plan launches on (torch's
    current stream)."""
    import torch

    for _ in range(2):
        plan.force(pose, t=t, want_wrench=False)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plan.force(pose, t=t, want_wrench=False)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def _roofline(fpp, pairs, k_ms, launch, traffic, kernel):
    achieved = fpp * pairs / (k_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic, "kernel": kernel, "ms_per_launch": k_ms,
            "pairs_per_launch": pairs, "flops_per_pair": fpp, "pairs_per_s": pairs / (k_ms * 1e-3),
            "launch": launch, "peak_unpacked": PEAK_FP32_UNPACKED_TFLOPS,
            "frac_unpacked": achieved / PEAK_FP32_UNPACKED_TFLOPS}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the scan, batch, adjoint, mixed ... legs")
    ap.add_argument("--legs", default="scene,scan,batch,adjoint,force_law,pyramid,vector",
                    help="comma-separated extra legs to run (default: all)")
    ap.add_argument("--autotune", action="store_true",
                    help="re-tune the force kernel launch shape instead of loading the committed tile table")
    ap.add_argument("--save-tiles", default="", help="write the tile table here after tuning")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (traffic-counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py measures one GPU only: the registration hot path runs on a single "
                                   "MI355X (multi-GPU sharding is a design note, not implemented)",
                          "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    if args.calibrate_copy:
        n = 64 * 1024 * 1024       # float32 elements: 256 MiB read + 256 MiB written per copy
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": 4 * n, "bytes_written": 4 * n, "copies": 5}))
        return 0

    import paper_1902_01061_amd as sg
    from synth import config5

    pr = config5()
    E, k, p, g_mode = 100, 16, 1.0, 1
    prm = sg.Params(p=p, g_mode=g_mode, k=k, E=E)
    M, N = pr.M, pr.N
    log(f"workload: depth-frame scene, template {M} x reference {N}, k={k}, E={E}, p={p}, g=a a s")
    ctx = sg.Context(0)
    tm, rf = sg.Cloud(pr.tmpl), sg.Cloud(pr.ref)
    ident = sg.pose_identity()
    pose = ident.clone()

    a_t, mom_t = ctx.descriptors(tm, k)
    a_r, mom_r = ctx.descriptors(rf, k)
    if args.autotune or not os.path.exists(TILES):
        tuned, tuned_ms = ctx.autotune(tm, a_t, rf, a_r, mom_t, mom_r, prm, reps=5)
        log(f"autotuned force kernel launch: R={tuned[0]} blocks/CU={tuned[1]} variant={tuned[2]} ({tuned_ms:.4f} ms)")
        if args.save_tiles:
            ctx.save_tiles(args.save_tiles)
        launch = {"R": tuned[0], "blocks_per_cu": tuned[1], "variant": tuned[2]}
    else:
        ctx.load_tiles(TILES)
        log(f"tile table loaded from {os.path.relpath(TILES, ROOT)}")
        launch = _launch_of(TILES, M, N, p)
    for w in range(args.warmup):
        pose.copy_(ident)
        ctx.register(tm, rf, prm, pose=pose)
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        pose.copy_(ident)
        ctx.register(tm, rf, prm, pose=pose)
        log(f"timed registration {s + 1}/{args.steps} launched")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"timed {args.steps} registrations: {dt:.3f} s")
    ms_per_step = dt / args.steps * 1e3
    value = M * N * E * args.steps / dt
    pose_err = _pose_err(sg, pose, pr)
    nn_rmse = float(ctx.residual(tm, rf, pose).item())

    # dominant kernel: the all-pairs force kernel alone, on the final pose
    plan = sg.Plan(ctx, tm, a_t, rf, a_r, mom_t, mom_r, prm)
    k_ms = _kernel_ms(plan, pose, E - 1, args.kernel_reps)
    plan.close()
    roof = _roofline(FLOPS_PER_PAIR[1.0], M * N, k_ms, launch, _traffic(launch, M, N, p), "force_kernel (p = 1)")
    log(f"force kernel: {k_ms:.4f} ms/launch, {roof['pairs_per_s']:.3e} pairs/s, {roof['achieved']:.2f} TFLOP/s")
    # the same kernel with the p = 2 distance law (one log2 + one exp2 per pair)
    prm2 = sg.Params(p=2.0, g_mode=g_mode, k=k, E=E)
    plan2 = sg.Plan(ctx, tm, a_t, rf, a_r, mom_t, mom_r, prm2)
    k2_ms = _kernel_ms(plan2, pose, E - 1, max(3, args.kernel_reps // 2))
    plan2.close()
    launch2 = _launch_of(TILES, M, N, 2.0) if os.path.exists(TILES) else None
    roof2 = _roofline(FLOPS_PER_PAIR[2.0], M * N, k2_ms, launch2, _traffic(launch2, M, N, 2.0),
                      "force_kernel (p = 2, r-form)")
    log(f"force kernel p=2: {k2_ms:.4f} ms/launch, {roof2['pairs_per_s']:.3e} pairs/s")

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
        "config": {"workload": f"depth-frame scene registration: reference {N} points (640x480 frame of a 5x3x4 m "
                               f"room with 20 boxes, depth noise 0.001 z^2), template {M} points (one box removed, "
                               f"two added, camera turned 30 deg), k={k} curvature, p={p:g}, g=a a s (eq. 10), "
                               f"{E} iterations",
                   "M": M, "N": N, "iterations": E, "k": k, "p": p, "g_mode": g_mode},
        "ms_per_registration": ms_per_step,
        "pose_rmse_over_diameter": pose_err,
        "nn_rmse": nn_rmse,
        "roofline": roof,
        "roofline_rform": roof2,
    }
    out.update(_reference_errors(pr))
    legs = set() if args.no_extras else set(args.legs.split(","))
    if "scene" in legs:
        out["scene"] = extra_scene(sg, ctx, pr, dt / args.steps, pose)
        log(f"scene: mixed {out['scene']['mixed']['ms_per_registration']:.1f} ms, "
            f"pose-independent sums {out['scene']['pose_independent_sums']['ms_per_registration']:.1f} ms")
    if "scan" in legs:
        out["scan"] = extra_scan(sg, ctx, args.steps, 20)
        log(f"scan: fp32 {out['scan']['fp32']['ms_per_registration']:.1f} ms, "
            f"{out['scan']['rows_with_force_at_t0']} rows with a force")
    if "batch" in legs:
        out["batch"] = extra_batch(sg, ctx)
        log(f"batch: {out['batch']['ms_per_batch']:.1f} ms, pose-independent sums "
            f"{out['batch']['pose_independent_sums']['ms_per_batch']:.1f} ms")
    if "adjoint" in legs:
        out["adjoint"] = extra_adjoint(sg, ctx)
        log(f"adjoint: fwd {out['adjoint']['fwd_ms']:.3f} ms, bwd {out['adjoint']['bwd_ms']:.3f} ms")
    if "force_law" in legs:
        out["force_law"] = extra_force_law(sg, ctx, 300, 24)
        log(f"force law: workload pose error p=1 {out['force_law']['workload']['shape_p1']['pose_rmse_over_diameter']:.2e}"
            f", gravitational {out['force_law']['workload']['gravitational_p-2']['pose_rmse_over_diameter']:.2e}")
    if "pyramid" in legs:
        out["pyramid"] = extra_pyramid(sg, ctx, 300, 24)
        log(f"pyramid: radius descriptors {out['pyramid']['radius_descriptors']['ms']:.3f} ms, registration "
            f"{out['pyramid']['pyramid']['ms_per_registration']:.1f} ms")
    if "vector" in legs:
        out["vector"] = extra_vector(sg, ctx, 300, 24)
        log(f"vector descriptors: split f16 {out['vector']['split_f16']['ms_per_registration']:.1f} ms, "
            f"fp32 {out['vector']['fp32']['ms_per_registration']:.1f} ms, pose-independent sums "
            f"{out['vector']['split_f16_pose_independent_sums']['ms_per_registration']:.1f} ms per registration")
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(pr, E, k, args.cpu_seconds, g_mode=g_mode)
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
