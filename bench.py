#!/usr/bin/env python3
"""Throughput of the MI355X Gaussian-splatting rasterizer on one GPU.

Step (timed): one mapping iteration on the 640x480 workload with 200k
Gaussians - projection, depth sort and tile binning, forward compositing,
L1 loss (colour 1, depth 0.5) and the full backward to the Gaussian
parameters - replayed as one captured graph, as an optimiser runs it over
fixed keyframes.  `value` = pixels per second of that step (Mpix/s).  The
same step through the eager entry points is timed too; its per-kernel HIP
event timings (the library brackets each kernel on its launch stream) give
the roofline of the dominant kernel.
Alongside: candidate views scored per second, batched (one persistent launch /
captured graph) vs plain (per-view launches), on the 64-view 320x240 workload
(500k Gaussians) and the 256-view uneven workload (2M Gaussians); the roofline
of the dominant kernel; and the FP64 oracle timed on the host cores.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "render+backward Mpix/s and candidate views scored/s, batched vs plain, 1 GPU"

# Algorithmic work per unit:
#  forward compositing: 20 FP32 VALU operations per contributing pixel-splat pair;
#  backward compositing: 55 FP32 VALU operations per contributing pair.
OPS_PER_PAIR = {"render": 20.0, "render_backward": 55.0}
# FP32 vector peak in lane-operations per second: 256 CUs x 4 SIMDs x 32 lanes
# per cycle (a wave64 instruction every 2 cycles) x 2.4 GHz = 78.6e12, i.e. the
# 157.3 TFLOP/s FP32 vector figure counting a fused multiply-add as one operation
ALU_PEAK_OPS = 256 * 4 * 32 * 2.4e9
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes, scaled by
# the counter readings of a plain 256 MiB copy (fetch x2.0, write x1.0); valid
# only for the kernel source they were taken on (sha256 of rtg_kernels.hip).
TRAFFIC = {
    "render_backward": (14164.1 * 2.0 * 1024 + 26269.2 * 1024,
                        "8688c1a69e5f0abad5b50452373e61095f5155f9e2f29d933a93c772b0acf344"),
    "render": (11344.3 * 2.0 * 1024 + 8400.0 * 1024,
               "8688c1a69e5f0abad5b50452373e61095f5155f9e2f29d933a93c772b0acf344"),
}


def kernel_source_sha():
    import hashlib
    path = os.path.join(ROOT, "paper_2409_18122_amd", "csrc", "rtg_kernels.hip")
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-scoring", action="store_true", help="skip the view-scoring workloads")
    ap.add_argument("--no-uneven", action="store_true", help="skip the 256-view uneven scoring workload")
    ap.add_argument("--no-keyframes", action="store_true", help="skip the 8-keyframe 1280x720 mapping workload")
    ap.add_argument("--no-collision", action="store_true", help="skip the 3M-Gaussian collision-check workload")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--tile", type=str, default="16x16")
    ap.add_argument("--sweep-tiles", action="store_true", help="also time the step at every tile shape")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the rasterizer "
              "path has no multi-GPU component in this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import scenes
    from paper_2409_18122_amd import raster

    tw, th = (int(x) for x in args.tile.split("x"))
    S = dict(scenes.DEFAULT_SETTINGS, tile_w=tw, tile_h=th)
    ctx = raster.Context(0)
    dev = torch.device("cuda:0")

    if args.calibrate_copy:
        a = torch.ones(64 << 20, device=dev, dtype=torch.float32)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 256 MiB device-to-device copies")
        del a, b

    # ------------------------------------------------------- mapping step
    log("setup: 640x480 mapping workload, 200k Gaussians")
    g_np, cams, tgt_np = scenes.config2()
    g = raster.to_device(g_np)
    tg = raster.to_device(tgt_np)
    target, tf = raster.render(ctx, tg, cams, S, want=("rgb", "depth"))
    tf.close()
    P = cams[0]["width"] * cams[0]["height"]
    grads = {k: torch.zeros_like(g[k]) for k in raster.GRAD_KEYS}

    def step():
        f = raster.Frame(ctx, g, cams, S)
        f.bin_sort()
        out = f.render(("rgb", "depth"))
        loss, d_rgb, d_dep = f.loss(out["rgb"], out["depth"], target["rgb"], target["depth"], 0.5)
        f.backward(d_rgb, d_dep, grads=grads)
        return f

    for _ in range(args.warmup):
        step().close()
    torch.cuda.synchronize()
    f = step()
    stats = f.stats()
    f.close()
    raster.timing_reset(ctx)
    raster.timing_enable(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step().close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    raster.timing_enable(ctx, False)
    kern = raster.timing_read(ctx)
    ms_eager = (t1 - t0) * 1e3 / args.steps
    log(f"eager mapping step {ms_eager:.3f} ms -> {P / (ms_eager * 1e-3) / 1e6:.1f} Mpix/s; stats {stats}")

    # the same step captured once and replayed (the optimiser's inner loop)
    mg = raster.MapGraph(ctx, g, cams, target["rgb"], target["depth"], 0.5, S, grads=grads)
    for _ in range(args.warmup):
        mg.launch()
    torch.cuda.synchronize()
    assert mg.status(), "mapping graph capacity overflow"
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mg.launch()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert mg.status(), "mapping graph capacity overflow"
    mg.close()
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = P / (ms_step * 1e-3) / 1e6
    log(f"captured mapping step {ms_step:.3f} ms -> {value:.1f} Mpix/s")

    # the same captured step with the full loss of eq. (4) (L1 depth + 0.4 L1 colour
    # + 0.1 (1 - SSIM)), and the SSIM loss kernels alone (forward + backward)
    mgs = raster.MapGraph(ctx, g, cams, target["rgb"], target["depth"], 1.0, S, grads=grads,
                          lambda1=0.4, lambda2=0.1)
    for _ in range(args.warmup):
        mgs.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        mgs.launch()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert mgs.status(), "mapping graph capacity overflow"
    mgs.close()
    ms_eq4 = (t1 - t0) * 1e3 / args.steps
    fl = raster.Frame(ctx, g, cams, S)
    fl.bin_sort()
    img = fl.render(("rgb", "depth"))
    for _ in range(3):
        fl.loss_ssim(img["rgb"], img["depth"], target["rgb"], target["depth"], 1.0, 0.4, 0.1)
    e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
    e0.record()
    for _ in range(20):
        fl.loss_ssim(img["rgb"], img["depth"], target["rgb"], target["depth"], 1.0, 0.4, 0.1)
    e1.record()
    torch.cuda.synchronize()
    fl.close()
    ssim_us = e0.elapsed_time(e1) / 20 * 1e3
    eq4 = {"ms_per_step": round(ms_eq4, 4), "mpix_per_s": round(P / (ms_eq4 * 1e-3) / 1e6, 1),
           "loss_ssim_us": round(ssim_us, 1)}
    log(f"captured mapping step with eq. (4): {eq4}")
    log("kernel ms per step: " + ", ".join(f"{k}={v[0] / args.steps:.3f}" for k, v in kern.items() if v[1]))

    if args.sweep_tiles:
        for tile in ((8, 8), (16, 16), (32, 8)):
            S2 = dict(S, tile_w=tile[0], tile_h=tile[1])

            def step2():
                f = raster.Frame(ctx, g, cams, S2)
                f.bin_sort()
                out = f.render(("rgb", "depth"))
                loss, d_rgb, d_dep = f.loss(out["rgb"], out["depth"], target["rgb"], target["depth"], 0.5)
                f.backward(d_rgb, d_dep, grads=grads)
                return f
            for _ in range(2):
                step2().close()
            raster.timing_reset(ctx)
            raster.timing_enable(ctx, True)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            for _ in range(10):
                step2().close()
            torch.cuda.synchronize()
            tb = time.perf_counter()
            raster.timing_enable(ctx, False)
            kk = raster.timing_read(ctx)
            log(f"tile {tile}: {(tb - ta) * 100:.3f} ms/step; " +
                ", ".join(f"{k}={v[0] / 10:.3f}" for k, v in kk.items() if v[1]))

    # roofline of the dominant compositing kernel
    per_step = {k: v[0] / max(v[1], 1) for k, v in kern.items()}
    dom = max(("render", "render_backward"), key=lambda k: per_step[k])
    avg_ms = per_step[dom]
    ops = OPS_PER_PAIR[dom] * stats["contrib_pairs"]
    achieved = ops / (avg_ms * 1e-3) / 1e12
    roof = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3),
            "peak": round(ALU_PEAK_OPS / 1e12, 2), "unit": "TOP/s", "frac": round(achieved * 1e12 / ALU_PEAK_OPS, 4),
            "traffic": (TRAFFIC[dom][0] if dom in TRAFFIC and TRAFFIC[dom][1] == kernel_source_sha() else None),
            "avg_ms": round(avg_ms, 4), "units": stats["contrib_pairs"],
            "ops_per_unit": OPS_PER_PAIR[dom]}

    # ------------------------------------------------- 8 keyframes, 1M Gaussians
    keyframes = None
    if not args.no_keyframes:
        log("setup: 8 keyframes 1280x720, 1M Gaussians (tile chosen by the autotuner)")
        g4_np, cams4, t4_np = scenes.config4()
        g4 = raster.to_device(g4_np)
        t4 = raster.to_device(t4_np)
        S4 = raster.autotune(ctx, g4, cams4, 1, S)
        timg4, tf4 = raster.render(ctx, t4, cams4, S4, want=("rgb", "depth"))
        tf4.close()
        grads4 = {k: torch.zeros_like(g4[k]) for k in raster.GRAD_KEYS}
        mg4 = raster.MapGraph(ctx, g4, cams4, timg4["rgb"], timg4["depth"], 0.5, S4, grads=grads4)
        for _ in range(2):
            mg4.launch()
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            mg4.launch()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        assert mg4.status(), "keyframe mapping graph capacity overflow"
        mg4.close()
        P4 = sum(c["width"] * c["height"] for c in cams4)
        keyframes = {"ms_per_step": round(dt * 1e3, 3), "mpix_per_s": round(P4 / dt / 1e6, 1),
                     "tile": f"{S4['tile_w']}x{S4['tile_h']}", "batch": S4["batch"], "pixels": P4}
        log(f"8 keyframes: {keyframes}")
        del g4, t4, grads4

    # ------------------------------------------------------- view scoring
    views = {}
    if not args.no_scoring:
        log("setup: 64-view 320x240 scoring workload, 500k Gaussians")
        g3_np, cams3 = scenes.config3()
        g3 = raster.to_device(g3_np)
        for persistent, name in ((True, "batched"), (False, "plain")):
            raster.score_views(ctx, g3, cams3, S, persistent=persistent)
            torch.cuda.synchronize()
            reps = 5
            t0 = time.perf_counter()
            for _ in range(reps):
                raster.score_views(ctx, g3, cams3, S, persistent=persistent)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            views[f"64x320x240_{name}"] = round(len(cams3) / dt, 1)
            log(f"64 views {name}: {dt * 1e3:.2f} ms")
        del g3
    bookkeeping = None
    if not args.no_scoring and not args.no_uneven:
        log("setup: 256-view uneven scoring workload, 2M Gaussians")
        g5_np, cams5 = scenes.config5()
        g5 = raster.to_device(g5_np)
        gr = raster.ScoreGraph(ctx, g5, 256, 640, 480, S, probe=cams5)
        gr.launch(cams5)
        torch.cuda.synchronize()
        assert gr.status(), "graph capacity overflow"
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            gr.launch(cams5)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        assert gr.status()
        views["256_uneven_graph"] = round(len(cams5) / dt, 1)
        log(f"256 views graph: {dt * 1e3:.2f} ms")
        gr.close()
        # the binary-J trace (sum of u over contributing Gaussians), same pipeline
        grb = raster.ScoreGraph(ctx, g5, 256, 640, 480, S, probe=cams5, mode="binary")
        grb.launch(cams5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            grb.launch(cams5)
        torch.cuda.synchronize()
        dtb = (time.perf_counter() - t0) / reps
        assert grb.status(), "graph capacity overflow"
        views["256_uneven_graph_binary_j"] = round(len(cams5) / dtb, 1)
        grb.close()
        f5 = raster.Frame(ctx, g5, cams5, S)
        f5.bin_sort()
        f5.render(("alpha",))
        st5 = f5.stats()
        f5.close()
        log(f"256-view frame stats: {st5}")
        raster.score_views(ctx, g5, cams5, S, persistent=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        raster.score_views(ctx, g5, cams5, S, persistent=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        views["256_uneven_batched_eager"] = round(len(cams5) / dt, 1)
        t0 = time.perf_counter()
        raster.score_views(ctx, g5, cams5, S, persistent=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        views["256_uneven_plain"] = round(len(cams5) / dt, 1)
        log(f"256 views: {views}")

        # ------------------------- uncertainty bookkeeping and region utility
        # over the 2M-Gaussian map: u = |mu_k - mu_{k-1}| with retention, then
        # the mean uncertainty of 2.5 m regions; algorithmic bytes per
        # Gaussian: 28 read + 4 written, and 16 read
        n5 = int(g5["opacity"].shape[0])
        prev = g5["means"] + 0.01 * torch.randn_like(g5["means"])
        prev[:, ::3] = g5["means"][:, ::3]
        u5 = torch.rand(n5, device=dev)
        box = [-10.0, -10.0, 0.0, 10.0, 10.0, 4.0]
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        for _ in range(2):
            raster.uncertainty_update(ctx, prev, g5["means"], u5, out=u5)
            raster.region_utility(ctx, g5["means"], u5, box, 2.5)
        reps = 20
        e0.record()
        for _ in range(reps):
            raster.uncertainty_update(ctx, prev, g5["means"], u5, out=u5)
        e1.record()
        for _ in range(reps):
            raster.region_utility(ctx, g5["means"], u5, box, 2.5)
        e2.record()
        torch.cuda.synchronize()
        t_upd = e0.elapsed_time(e1) / reps * 1e-3
        t_reg = e1.elapsed_time(e2) / reps * 1e-3
        bookkeeping = {"gaussians": n5,
                       "update_us": round(t_upd * 1e6, 2), "update_GBps": round(32.0 * n5 / t_upd / 1e9, 1),
                       "region_us": round(t_reg * 1e6, 2), "region_GBps": round(16.0 * n5 / t_reg / 1e9, 1),
                       "regions": int(np.prod(raster.region_grid(box, 2.5)))}
        log(f"bookkeeping: {bookkeeping}")

    # ------------------------------------------------------- collision check
    # 3M Gaussians over a 40 m x 40 m lot; one 5 m motion primitive of 129
    # points, and a tree layer of 64 such primitives; every point against
    # every Gaussian.  The pair loop issues 15 VALU instructions per pair.
    collision = None
    if not args.no_collision:
        glot = scenes.lot_scene()
        gl = {k: torch.as_tensor(glot[k]).to(dev) for k in ("means", "log_scales")}
        nl = int(glot["means"].shape[1])
        collision = {"gaussians": nl, "r_robot": 0.25, "lambda_g": 3.0}
        for name, n_paths in (("1x129", 1), ("64x129", 64)):
            pl = torch.as_tensor(scenes.path_points(n_paths, 7)).to(dev)
            npt = int(pl.shape[1])
            for _ in range(2):
                raster.collision_check(ctx, gl, pl, 0.25, 3.0)
            reps = 10 if n_paths > 1 else 50
            e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
            e0.record()
            for _ in range(reps):
                hit, _ = raster.collision_check(ctx, gl, pl, 0.25, 3.0)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / reps * 1e-3
            pairs = float(nl) * npt
            collision[name] = {"points": npt, "us": round(t * 1e6, 1), "Gpairs_per_s": round(pairs / t / 1e9, 1),
                               "alu_frac": round(pairs * 15 / t / ALU_PEAK_OPS, 3),
                               "collisions": int(hit.sum().item())}
        log(f"collision: {collision}")

    # ------------------------------------------------------- CPU baseline
    cpu = None
    if not args.no_cpu:
        import oracle
        threads = min(os.cpu_count() or 1, 16)
        oracle.set_threads(threads)
        log(f"oracle baseline on {threads} threads")
        rt = oracle.render(tgt_np, cams[0], S)
        trgb = rt["rgb"].astype(np.float32)
        tdep = rt["depth"].astype(np.float32)
        n = 0
        t0 = time.perf_counter()
        while True:
            r = oracle.render(g_np, cams[0], S)
            _, gr_, gd_ = oracle.loss(r["rgb"], r["depth"], trgb, tdep, 0.5)
            oracle.adjoint(g_np, cams[0], S, g_rgb=gr_, g_depth=gd_)
            n += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        dt = time.perf_counter() - t0
        cpu = {"value": round(n * P / dt / 1e6, 4), "unit": "Mpix/s", "cores": oracle.max_threads(),
               "kind": "oracle",
               "sample": f"{n} full 640x480 mapping steps (render + loss + adjoint) of the 200k-Gaussian "
                         f"workload, FP64, {dt:.1f} s"}
        log(f"oracle: {cpu}")

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "ms_per_step_eager": round(ms_eager, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mapping step: 200k Gaussians, one 640x480 RGB-D frame (fx=fy=525), "
                               "forward + L1 RGB + 0.5 L1 depth + backward, captured as one graph per "
                               "iteration",
                   "tile": f"{tw}x{th}", "gaussians": 200000, "pixels": P},
        "roofline": roof,
        "cpu_baseline": cpu,
        "views_per_s": views,
        "mapping_step_eq4_loss": eq4,
        "keyframes_8x1280x720": keyframes,
        "bookkeeping_2M": bookkeeping,
        "collision_3M": collision,
        "kernel_ms_per_step_eager": {k: round(v[0] / args.steps, 4) for k, v in kern.items() if v[1]},
        "frame_stats": stats,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
