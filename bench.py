#!/usr/bin/env python3
"""Throughput of the MI355X Gaussian-splatting rasterizer on one GPU.

Step (timed, `value`): one mapping iteration over 8 keyframes of 1280x720
sharing a map of 1M Gaussians - projection, depth sort and tile binning,
forward compositing, L1 loss (colour 1, depth 0.5) summed over the frames,
and the full backward into shared gradients - replayed as one captured graph,
as an optimiser iterates over fixed keyframes.  The tile comes from the
autotuner.  `value` = pixels per second of that step (Mpix/s).  The same step
through the eager entry points gives, from the library's per-kernel HIP
events on the launch stream, the roofline of the dominant kernel.

Alongside (each a hipEvent median over replays after warm-up): the 640x480
mapping step (200k Gaussians, L1 and the full eq. (4) loss), the 128x96
forward render (2k Gaussians), candidate views scored per second, batched (one
persistent launch, and a captured graph) against plain (per-view launches),
on 64 views of 320x240 (500k Gaussians) and 256 uneven views (2M Gaussians,
with the scoring kernel's roofline and the binning kernels' HBM rates), the
paper's non-rendering view utility of eq. (8) with its thresholds and the
trajectory selection of eq. (10), the uncertainty bookkeeping, the collision
check, and the FP64 oracle timed on the host cores.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import statistics
import sys
import tempfile
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "render+backward Mpix/s and candidate views scored/s, batched vs plain, 1 GPU"

# Algorithmic work per unit, FP32 VALU operations per contributing
# pixel-splat pair, counted on the method's arithmetic:
#  alpha: offset (2), whitened offset (3), squared norm (2), exp2, times
#   opacity, clamp to alpha_max = 10; the alpha_min test = 1;
#  forward: alpha and test (11), next transmittance, its T_min test, weight
#   (3), colour and depth accumulation (4) = 18;
#  backward: alpha and test (11), 1 - a and its reciprocal, T_i, weight (4),
#   gradient-weighted colour (4), dL/da (2), its running sum (1), colour and
#   depth gradients (4), opacity term and dL/dpower (3), the offset products
#   (2) and the five geometric sums (5) = 36;
#  scoring: alpha with the opacity inside the exponent (9), test (1), next
#   transmittance, its test, weight, uncertainty accumulation (4) = 14.
OPS_PER_PAIR = {"render": 18.0, "render_backward": 36.0, "score": 14.0}
# FP32 vector peak in lane-operations per second: 256 CUs x 4 SIMDs x 32 lanes
# per cycle (a wave64 instruction every 2 cycles) x 2.4 GHz = 78.6e12, i.e. the
# 157.3 TFLOP/s FP32 vector figure counting a fused multiply-add as one operation
ALU_PEAK_OPS = 256 * 4 * 32 * 2.4e9
HBM_PEAK = 8.0e12

# HBM bytes per launch on the 8-keyframe step from rocprofv3 FETCH_SIZE /
# WRITE_SIZE passes, scaled by the counter readings of a plain 256 MiB copy
# (fetch x2.0, write x1.0); valid only for the kernel source they were taken on
# (sha256 of rtg_kernels.hip).
TRAFFIC = {
    "render_backward": (208829.0 * 2.0 * 1024 + 712236.0 * 1024,
                        "ff30b1a24fd69bfd0d4cb859a9073a5618f88bd7beecc9b1048a76a48d48022e"),
}

SECTIONS = ("c4", "c2", "c1", "c3", "c5", "utility", "bookkeeping", "collision")


def kernel_source_sha():
    import hashlib
    path = os.path.join(ROOT, "paper_2409_18122_amd", "csrc", "rtg_kernels.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def event_times(fn, reps, warm):
    """Per-call milliseconds by HIP events on torch's current stream (the
    library's launch stream), after `warm` untimed calls."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def med(ts):
    return float(statistics.median(ts))


def roof_alu(name, avg_ms, units, ops_per_unit):
    achieved = ops_per_unit * units / (avg_ms * 1e-3)
    return {"bound": "alu", "kernel": name, "achieved": round(achieved / 1e12, 3),
            "peak": round(ALU_PEAK_OPS / 1e12, 2), "unit": "TOP/s", "frac": round(achieved / ALU_PEAK_OPS, 4),
            "avg_ms": round(avg_ms, 4), "units": int(units), "ops_per_unit": ops_per_unit}


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable": usable, "model": model}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed replays of the headline step")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--reps", type=int, default=50, help="timed replays of every other workload")
    ap.add_argument("--only", type=str, default=",".join(SECTIONS),
                    help="comma-separated sections: " + ",".join(SECTIONS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-view (plain) scoring loops")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the rasterizer "
              "path has no multi-GPU component in this build.", file=sys.stderr)
        sys.exit(2)
    only = set(x.strip() for x in args.only.split(",") if x.strip())
    bad = only - set(SECTIONS)
    if bad:
        sys.exit(f"unknown sections {sorted(bad)}")

    import numpy as np
    import torch

    import scenes
    from paper_2409_18122_amd import raster

    S = dict(scenes.DEFAULT_SETTINGS)
    ctx = raster.Context(0)
    dev = torch.device("cuda:0")
    W, R = args.warmup, args.reps
    line = {"metric": METRIC}

    if args.calibrate_copy:
        a = torch.ones(64 << 20, device=dev, dtype=torch.float32)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 256 MiB device-to-device copies")
        del a, b

    def mapping_step_fn(g, cams, target, st, grads):
        def step():
            f = raster.Frame(ctx, g, cams, st)
            f.bin_sort()
            out = f.render(("rgb", "depth"))
            _, d_rgb, d_dep = f.loss(out["rgb"], out["depth"], target["rgb"], target["depth"], 0.5)
            f.backward(d_rgb, d_dep, grads=grads)
            return f
        return step

    def kernel_ms(step, n):
        """Library per-kernel event timings (ms per step) over n eager steps."""
        raster.timing_reset(ctx)
        raster.timing_enable(ctx, True)
        for _ in range(n):
            step().close()
        torch.cuda.synchronize()
        raster.timing_enable(ctx, False)
        k = raster.timing_read(ctx)
        return {name: (ms / n, cnt) for name, (ms, cnt) in k.items() if cnt}

    # ------------------------------------------------- headline: 8 keyframes
    headline = None
    if "c4" in only:
        log("setup: 8 keyframes 1280x720, 1M Gaussians (tile chosen by the autotuner)")
        g4_np, cams4, t4_np = scenes.config4()
        g4 = raster.to_device(g4_np)
        t4 = raster.to_device(t4_np)
        S4 = raster.autotune(ctx, g4, cams4, 1, S)
        timg4, tf4 = raster.render(ctx, t4, cams4, S4, want=("rgb", "depth"))
        tf4.close()
        del t4
        grads4 = {k: torch.zeros_like(g4[k]) for k in raster.GRAD_KEYS}
        P4 = sum(c["width"] * c["height"] for c in cams4)
        step4 = mapping_step_fn(g4, cams4, timg4, S4, grads4)
        for _ in range(3):
            step4().close()
        f = step4()
        stats4 = f.stats()
        f.close()
        kern4 = kernel_ms(step4, 10)
        log(f"8 keyframes eager kernels (ms/step): " + ", ".join(f"{k}={v[0]:.3f}" for k, v in kern4.items()))
        mg4 = raster.MapGraph(ctx, g4, cams4, timg4["rgb"], timg4["depth"], 0.5, S4, grads=grads4)
        for _ in range(W):
            mg4.launch()
        torch.cuda.synchronize()
        assert mg4.status(), "keyframe mapping graph capacity overflow"
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in evs:
            a.record()
            mg4.launch()
            b.record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        assert mg4.status(), "keyframe mapping graph capacity overflow"
        mg4.close()
        ms_step = (t1 - t0) * 1e3 / args.steps
        ev_ms = [a.elapsed_time(b) for a, b in evs]
        value = P4 / (ms_step * 1e-3) / 1e6
        log(f"8 keyframes captured step {ms_step:.3f} ms (event median {med(ev_ms):.3f}) -> {value:.1f} Mpix/s")
        roofs = {k: roof_alu(k, kern4[k][0], stats4["contrib_pairs"], OPS_PER_PAIR[k])
                 for k in ("render", "render_backward") if k in kern4}
        dom = max(roofs, key=lambda k: roofs[k]["avg_ms"])
        roof = dict(roofs[dom])
        tr = TRAFFIC.get(dom)
        roof["traffic"] = tr[0] if tr and tr[1] == kernel_source_sha() else None
        roof["other"] = {k: {"frac": v["frac"], "avg_ms": v["avg_ms"]} for k, v in roofs.items() if k != dom}
        headline = {"value": value, "ms_step": ms_step, "ev_median": med(ev_ms), "roof": roof,
                    "tile": f"{S4['tile_w']}x{S4['tile_h']}", "batch": S4["batch"], "pixels": P4,
                    "stats": stats4, "kern": {k: round(v[0], 4) for k, v in kern4.items()}}
        del g4, grads4, timg4

    # ---------------------------------------------------- 640x480 mapping step
    mapping = None
    if "c2" in only:
        log("setup: 640x480 mapping workload, 200k Gaussians")
        g_np, cams, tgt_np = scenes.config2()
        g = raster.to_device(g_np)
        target, tf = raster.render(ctx, raster.to_device(tgt_np), cams, S, want=("rgb", "depth"))
        tf.close()
        P = cams[0]["width"] * cams[0]["height"]
        grads = {k: torch.zeros_like(g[k]) for k in raster.GRAD_KEYS}
        step2 = mapping_step_fn(g, cams, target, S, grads)
        for _ in range(3):
            step2().close()
        f = step2()
        stats2 = f.stats()
        f.close()
        kern2 = kernel_ms(step2, 20)
        eager = med(event_times(lambda: step2().close(), R, W))
        mg = raster.MapGraph(ctx, g, cams, target["rgb"], target["depth"], 0.5, S, grads=grads)
        t_l1 = med(event_times(mg.launch, R, W))
        assert mg.status(), "mapping graph capacity overflow"
        mg.close()
        mgs = raster.MapGraph(ctx, g, cams, target["rgb"], target["depth"], 1.0, S, grads=grads,
                              lambda1=0.4, lambda2=0.1)
        t_eq4 = med(event_times(mgs.launch, R, W))
        assert mgs.status(), "mapping graph capacity overflow"
        mgs.close()
        roofs2 = {k: roof_alu(k, kern2[k][0], stats2["contrib_pairs"], OPS_PER_PAIR[k])
                  for k in ("render", "render_backward") if k in kern2}
        mapping = {"ms_per_step": round(t_l1, 4), "mpix_per_s": round(P / (t_l1 * 1e-3) / 1e6, 1),
                   "eager_ms_per_step": round(eager, 4),
                   "eq4_ms_per_step": round(t_eq4, 4), "eq4_mpix_per_s": round(P / (t_eq4 * 1e-3) / 1e6, 1),
                   "kernel_ms": {k: round(v[0], 4) for k, v in kern2.items()},
                   "alu_frac": {k: v["frac"] for k, v in roofs2.items()}, "frame_stats": stats2}
        log(f"640x480 mapping step: {mapping}")
        del g, grads, target

    # ----------------------------------------------------- 128x96 forward
    forward = None
    if "c1" in only:
        g1_np, cams1 = scenes.config1()
        g1 = raster.to_device(g1_np)

        def fwd1():
            out, f = raster.render(ctx, g1, cams1, S)
            f.close()
        t = med(event_times(fwd1, R, W))
        P1 = cams1[0]["width"] * cams1[0]["height"]
        forward = {"ms": round(t, 4), "mpix_per_s": round(P1 / (t * 1e-3) / 1e6, 2), "pixels": P1}
        log(f"128x96 forward: {forward}")

    # ------------------------------------------------------- view scoring
    views = {}
    scoring = {}
    if "c3" in only:
        log("setup: 64-view 320x240 scoring workload, 500k Gaussians")
        g3_np, cams3 = scenes.config3()
        g3 = raster.to_device(g3_np)
        for persistent, name in ((True, "batched"), (False, "plain")):
            if not persistent and args.no_plain:
                continue
            t = med(event_times(lambda: raster.score_views(ctx, g3, cams3, S, persistent=persistent), R, W))
            views[f"64x320x240_{name}"] = round(len(cams3) / (t * 1e-3), 1)
        gr3 = raster.ScoreGraph(ctx, g3, 64, 320, 240, S, probe=cams3)
        t = med(event_times(lambda: gr3.launch(cams3), R, W))
        assert gr3.status(), "graph capacity overflow"
        gr3.close()
        views["64x320x240_graph"] = round(len(cams3) / (t * 1e-3), 1)
        log(f"64 views: {views}")
        del g3

    g5 = cams5 = None
    if "c5" in only or "utility" in only or "bookkeeping" in only:
        log("setup: 2M-Gaussian map, 256 uneven views")
        g5_np, cams5 = scenes.config5()
        g5 = raster.to_device(g5_np)
    if "c5" in only:
        for mode, name in (("rendered", "256_uneven_graph"), ("binary", "256_uneven_graph_binary_j")):
            gr = raster.ScoreGraph(ctx, g5, 256, 640, 480, S, probe=cams5, mode=mode)
            t = med(event_times(lambda: gr.launch(cams5), R, W))
            assert gr.status(), "graph capacity overflow"
            gr.close()
            views[name] = round(len(cams5) / (t * 1e-3), 1)
        t = med(event_times(lambda: raster.score_views(ctx, g5, cams5, S, persistent=True), R, W))
        views["256_uneven_batched_eager"] = round(len(cams5) / (t * 1e-3), 1)
        if not args.no_plain:
            t = med(event_times(lambda: raster.score_views(ctx, g5, cams5, S, persistent=False), max(R // 5, 10), 2))
            views["256_uneven_plain"] = round(len(cams5) / (t * 1e-3), 1)
        f5 = raster.Frame(ctx, g5, cams5, S)
        f5.bin_sort()
        f5.render(("alpha",))
        st5 = f5.stats()
        f5.close()
        # library timers over eager batched calls: projection, depth sort,
        # binning and the persistent compositing kernel
        raster.timing_reset(ctx)
        raster.timing_enable(ctx, True)
        nrep = 10
        for _ in range(nrep):
            raster.score_views(ctx, g5, cams5, S, persistent=True)
        torch.cuda.synchronize()
        raster.timing_enable(ctx, False)
        k5 = {k: v[0] / nrep for k, v in raster.timing_read(ctx).items() if v[1]}
        n5 = int(g5["opacity"].shape[0])
        # algorithmic bytes per launch group (the method's own traffic):
        #  projection: read 44 B per Gaussian (mean, log-scale, quaternion,
        #   opacity), write a 40-byte record per visible (view, Gaussian) pair;
        #  depth sort: read and write a (key, value) pair per record;
        #  binning: write a (tile, record) pair per instance, read and write it
        #   once to sort it by tile, read its tile key to find the ranges
        alg = {"project": 44.0 * n5 + 40.0 * st5["records"], "depth_sort": 16.0 * st5["records"],
               "binning": (8.0 + 16.0 + 4.0) * st5["instances"]}
        hbm = {k: {"ms": round(k5[k], 4), "GBps": round(alg[k] / (k5[k] * 1e-3) / 1e9, 1),
                   "frac": round(alg[k] / (k5[k] * 1e-3) / HBM_PEAK, 3)} for k in alg if k in k5}
        scoring = {"roofline": roof_alu("score_persistent", k5["score"], st5["contrib_pairs"], OPS_PER_PAIR["score"]),
                   "hbm_groups": hbm, "frame_stats": st5,
                   "eager_kernel_ms": {k: round(v, 4) for k, v in k5.items()}}
        log(f"256 views: {views}; scoring {scoring}")

    # ----------------------------- the paper's own metric: eq. (8) and eq. (10)
    utility = None
    if "utility" in only:
        n5 = int(g5["opacity"].shape[0])
        lo_hi = raster.uncertainty_thresholds(ctx, g5["uncert"])
        t_thr = med(event_times(lambda: raster.uncertainty_thresholds(ctx, g5["uncert"]), R, W))
        # camera tables built once, as a planner holding its candidates would
        c5 = raster.make_cameras(cams5)
        t_vu = med(event_times(lambda: raster.view_utility(ctx, g5, c5, lo_hi, S), R, W))
        tcams, toff = scenes.trajectory_states(64, 8)
        tc = raster.make_cameras(tcams)
        off_dev = torch.as_tensor(toff).to(dev)

        def traj():
            u = raster.view_utility(ctx, g5, tc, lo_hi, S)
            return raster.trajectory_select(ctx, u["xi"], off_dev)
        t_tr = med(event_times(traj, R, W))
        # algorithmic bytes: thresholds read u twice (mean, then deviation);
        # the utility reads each Gaussian's mean and u once for all views
        utility = {"gaussians": n5,
                   "thresholds_us": round(t_thr * 1e3, 1),
                   "thresholds_GBps": round(8.0 * n5 / (t_thr * 1e-3) / 1e9, 1),
                   "view_utility_256_views_us": round(t_vu * 1e3, 1),
                   "views_per_s": round(256 / (t_vu * 1e-3), 1),
                   "gaussian_view_tests_per_s": round(256.0 * n5 / (t_vu * 1e-3), 1),
                   "view_utility_GBps": round(16.0 * n5 / (t_vu * 1e-3) / 1e9, 1),
                   "trajectories": 64, "states": len(tcams),
                   "eq10_select_us": round(t_tr * 1e3, 1)}
        log(f"utility: {utility}")

    bookkeeping = None
    if "bookkeeping" in only:
        # u = |mu_k - mu_{k-1}| with retention, then the mean uncertainty of
        # 2.5 m regions; algorithmic bytes per Gaussian: 28 read + 4 written,
        # and 16 read
        n5 = int(g5["opacity"].shape[0])
        prev = g5["means"] + 0.01 * torch.randn_like(g5["means"])
        prev[:, ::3] = g5["means"][:, ::3]
        u5 = torch.rand(n5, device=dev)
        box = [-10.0, -10.0, 0.0, 10.0, 10.0, 4.0]
        t_upd = med(event_times(lambda: raster.uncertainty_update(ctx, prev, g5["means"], u5, out=u5), R, W))
        t_reg = med(event_times(lambda: raster.region_utility(ctx, g5["means"], u5, box, 2.5), R, W))
        bookkeeping = {"gaussians": n5,
                       "update_us": round(t_upd * 1e3, 2), "update_GBps": round(32.0 * n5 / (t_upd * 1e-3) / 1e9, 1),
                       "region_us": round(t_reg * 1e3, 2), "region_GBps": round(16.0 * n5 / (t_reg * 1e-3) / 1e9, 1),
                       "regions": int(np.prod(raster.region_grid(box, 2.5)))}
        log(f"bookkeeping: {bookkeeping}")
    del g5

    # ------------------------------------------------------- collision check
    # 3M Gaussians over a 40 m x 40 m lot; one 5 m motion primitive of 129
    # points, and a tree layer of 64 such primitives; every point against
    # every Gaussian.  The pair loop issues 15 VALU instructions per pair.
    collision = None
    if "collision" in only:
        glot = scenes.lot_scene()
        gl = {k: torch.as_tensor(glot[k]).to(dev) for k in ("means", "log_scales")}
        nl = int(glot["means"].shape[1])
        collision = {"gaussians": nl, "r_robot": 0.25, "lambda_g": 3.0}
        for name, n_paths in (("1x129", 1), ("64x129", 64)):
            pl = torch.as_tensor(scenes.path_points(n_paths, 7)).to(dev)
            npt = int(pl.shape[1])
            t = med(event_times(lambda: raster.collision_check(ctx, gl, pl, 0.25, 3.0), R, W)) * 1e-3
            hit, _ = raster.collision_check(ctx, gl, pl, 0.25, 3.0)
            pairs = float(nl) * npt
            collision[name] = {"points": npt, "us": round(t * 1e6, 1), "Gpairs_per_s": round(pairs / t / 1e9, 1),
                               "alu_frac": round(pairs * 15 / t / ALU_PEAK_OPS, 3),
                               "collisions": int(hit.sum().item())}
        log(f"collision: {collision}")

    # ------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu and "c4" in only:
        import oracle
        info = cpu_info()
        tmp = tempfile.mkdtemp(prefix="rtgo_")
        try:
            flags = oracle.use_native_build(tmp)
        except Exception as e:  # no compiler: the in-tree build
            flags = f"in-tree -O2 build ({e.__class__.__name__})"
        threads = info["usable"]
        oracle.set_threads(threads)
        used = oracle.max_threads()
        log(f"oracle baseline: {used} threads ({info}), {flags}")
        g4_np, cams4, t4_np = scenes.config4()
        S4 = dict(S, tile_w=int(headline["tile"].split("x")[0]), tile_h=int(headline["tile"].split("x")[1]))

        def oracle_frame(c, roi=None):
            """Seconds of render + loss + adjoint of camera c (of a window when
            roi); the target image is rendered first, outside the timing, as
            the GPU step takes its targets ready-made."""
            rt = oracle.render(t4_np, c, S4, roi=roi)
            trgb, tdep = rt["rgb"].astype(np.float32), rt["depth"].astype(np.float32)
            t0 = time.perf_counter()
            r = oracle.render(g4_np, c, S4, roi=roi)
            _, gr, gd = oracle.loss(r["rgb"], r["depth"], trgb, tdep, 0.5)
            if roi is not None:  # the loss and its gradient only inside the window
                x0, y0, x1, y1 = roi
                m = np.zeros(gd.shape, bool)
                m[y0:y1, x0:x1] = True
                gr = gr * m[None]
                gd = gd * m
            oracle.adjoint(g4_np, c, S4, g_rgb=gr, g_depth=gd, tile=(S4["tile_w"], S4["tile_h"]))
            return time.perf_counter() - t0

        # all host threads: keyframes in order until cpu_seconds of timed work
        # (at least one)
        dt = 0.0
        px = 0
        nk = 0
        for c in cams4:
            dt += oracle_frame(c)
            px += c["width"] * c["height"]
            nk += 1
            if dt >= args.cpu_seconds:
                break
        # one thread: a 320x180 window in the middle of keyframe 0
        oracle.set_threads(1)
        roi = (480, 270, 800, 450)
        dt1 = oracle_frame(cams4[0], roi=roi)
        px1 = (roi[2] - roi[0]) * (roi[3] - roi[1])
        oracle.set_threads(threads)
        cpu = {"value": round(px / dt / 1e6, 4), "unit": "Mpix/s", "cores": used, "kind": "oracle",
               "sample": f"{nk} of the 8 1280x720 keyframes, each a full FP64 render + L1 loss + adjoint of "
                         f"the 1M-Gaussian map, {dt:.1f} s",
               "nproc": info["nproc"], "cpu_model": info["model"], "build": flags,
               "one_thread": {"value": round(px1 / dt1 / 1e6, 5), "unit": "Mpix/s",
                              "sample": f"a 320x180 window of keyframe 0 (projection and sort of all 1M "
                                        f"Gaussians included), {dt1:.1f} s"}}
        log(f"oracle: {cpu}")
        # the other workloads, bounded samples on all threads
        extra = {}
        if "c2" in only:
            g_np, cams, tgt_np = scenes.config2()
            t0 = time.perf_counter()
            r = oracle.render(g_np, cams[0], S)
            rt = oracle.render(tgt_np, cams[0], S)
            _, gr, gd = oracle.loss(r["rgb"], r["depth"], rt["rgb"].astype(np.float32),
                                    rt["depth"].astype(np.float32), 0.5)
            oracle.adjoint(g_np, cams[0], S, g_rgb=gr, g_depth=gd)
            dt = time.perf_counter() - t0
            extra["mapping_640x480_mpix_per_s"] = round(307200 / dt / 1e6, 4)
        if "c1" in only:
            g1_np, cams1 = scenes.config1()
            t0 = time.perf_counter()
            n = 0
            while time.perf_counter() - t0 < 1.0:
                oracle.render(g1_np, cams1[0], S)
                n += 1
            extra["forward_128x96_mpix_per_s"] = round(n * 12288 / (time.perf_counter() - t0) / 1e6, 4)
        if "c3" in only:
            g3_np, cams3 = scenes.config3()
            t0 = time.perf_counter()
            oracle.score(g3_np, cams3[:4], S)
            extra["score_64x320x240_views_per_s"] = round(4 / (time.perf_counter() - t0), 3)
        if "c5" in only:
            g5_np, cams5 = scenes.config5()
            pick = []
            for w in (160, 320, 640):
                pick.append(next(c for c in cams5 if c["width"] == w))
            t0 = time.perf_counter()
            oracle.score(g5_np, pick, S)
            extra["score_256_uneven_views_per_s"] = round(3 / (time.perf_counter() - t0), 3)
            extra["score_256_uneven_sample"] = "one view of each resolution"
        cpu["other_workloads"] = extra
        log(f"oracle, other workloads: {extra}")

    if headline is not None:
        line.update({
            "value": round(headline["value"], 2), "unit": "Mpix/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(headline["ms_step"], 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "mapping step over 8 keyframes of 1280x720 (fx=fy=1050) sharing a map of "
                                   "1M Gaussians: projection, depth sort, tile binning, forward, L1 RGB + "
                                   "0.5 L1 depth loss summed over the frames, backward into shared gradients; "
                                   "one captured graph per iteration",
                       "tile": headline["tile"], "batch": headline["batch"], "gaussians": 1000000,
                       "keyframes": 8, "pixels": headline["pixels"]},
            "roofline": headline["roof"],
            "cpu_baseline": cpu,
            "ms_per_step_event_median": round(headline["ev_median"], 4),
            "kernel_ms_per_step_eager": headline["kern"],
            "frame_stats": headline["stats"],
        })
    line.update({
        "mapping_640x480": mapping,
        "forward_128x96": forward,
        "views_per_s": views,
        "scoring_256_uneven": scoring or None,
        "view_utility_eq8_eq10": utility,
        "bookkeeping_2M": bookkeeping,
        "collision_3M": collision,
    })
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
