#!/usr/bin/env python3
"""Throughput and latency of the coarse-to-fine visual-hull path on one MI355X.

One step is one frame of the volleyball-like workload: 16 cameras 1920x1080
(f in [1800, 2400] px) around an 18 x 9 x 4 m court, 12 players (unions of 5
ellipsoids), coarse lattice 100 mm (180 x 90 x 40), fine lattice 10 mm inside
the ROIs.  The step runs every stage of the path as one HIP graph: silhouette
packing, coarse carving, 26-connected labelling with the size filter and ROI
boxes, fine carving of all ROIs in one persistent launch, crossing-edge
compaction and exit-point bisection (8 steps).  The uint8 silhouettes of
--frames distinct synthetic frames are resident in HBM before timing starts;
steps cycle through them.

Metric: fine voxels carved per second of whole-frame time (sum of the ROI
lattice sizes over the timed frames / wall time of the timed loop), plus
per-frame latency p50/p99 from HIP events around each frame.

Prints ONE JSON line.  --gpus above 1 exits with a message: this path runs
on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = ("volleyball-like frame: 16 cams 1920x1080, 12 players x 5 ellipsoids, 18x9x4 m, "
            "coarse 100 mm (180x90x40), fine 10 mm in ROIs, 8-step edge bisection")
METRIC = "fine voxels carved/s + frame latency p50/p99 (16 cams 1080p, 12 ROIs)"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed frames (the paper averages 200)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--frames", type=int, default=8, help="distinct synthetic frames cycled")
    ap.add_argument("--stage-reps", type=int, default=20, help="eager runs per frame for the stage split")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU-baseline time budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fine-tile", default="64x4", help="TXxTZ of the fine carve")
    return ap.parse_args()


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, np.float64), q))


def cpu_baseline(frames, budget_s):
    """The oracle as it stands, on the same frames, until the budget is spent."""
    import oracle
    done_vox, spent, n, tests = 0, 0.0, 0, {}
    while spent < budget_s and n < 2000:
        sc = frames[n % len(frames)]
        t0 = time.perf_counter()
        r = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims, sc.t_np,
                         sc.t_nb, sc.n_steps)
        spent += time.perf_counter() - t0
        done_vox += r.fine_voxels
        tests[n % len(frames)] = (r.fine_voxels, r.tests_fine)
        n += 1
    return {"value": done_vox / spent, "unit": "fine voxels/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{n} whole volleyball-like frames (same inputs as the GPU steps), "
                      f"{spent:.1f} s of oracle time on host CPU"}, tests


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this path runs on one GPU; multi-GPU runs are not part of this build. "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import scenes
    import paper_1903_11785_amd as fvv

    torch.cuda.set_device(0)
    frames = [scenes.make_scene(scenes.CFG_VOLLEYBALL, f) for f in range(args.frames)]
    sc0 = frames[0]
    N, H, W = sc0.masks.shape
    coarse = fvv.Grid(origin=tuple(sc0.origin), h=sc0.hc, lo=(0, 0, 0), dims=sc0.coarse_dims)
    max_rois, max_fine, max_points = 256, 1 << 26, 1 << 22
    ctx = fvv.Context(max_cams=N, max_w=W, max_h=H, max_coarse=coarse.size, max_fine=max_fine,
                      max_rois=max_rois, max_points=max_points, max_jobs=max_rois)
    tx, tz = (int(v) for v in args.fine_tile.split("x"))
    params = fvv.frame_params(sc0.P32, W, H, coarse, sc0.hc_um, sc0.hf_um, sc0.t_np, sc0.t_nb,
                              sc0.n_steps, coarse_tile=fvv.tile(64, 1), fine_tile=fvv.tile(tx, tz))
    masks = [torch.from_numpy(sc.masks).cuda() for sc in frames]
    sils = torch.empty((N, H, (W + 31) // 32), dtype=torch.int32, device="cuda")
    bufs = fvv.FrameBuffers(coarse, max_rois, max_fine, max_points)

    # per-frame work (from one eager run each) and the per-stage split
    fine_vox, rois, points = [], [], []
    stage_ms = {s: [] for s in fvv.STAGES}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(fvv.FRAME_EVENTS)]
    for f, m in enumerate(masks):
        for rep in range(max(1, args.stage_reps)):
            ctx.frame(params, sils, bufs, masks=m, events=ev)
            torch.cuda.synchronize()
            if rep > 0:
                for i, s in enumerate(fvv.STAGES):
                    stage_ms[s].append(ev[i].elapsed_time(ev[i + 1]))
        if ctx.check() != fvv.FVV_OK:
            raise RuntimeError("frame exceeded a capacity")
        c = bufs.counts.cpu().numpy()
        rois.append(int(c[0]))
        fine_vox.append(int(c[1]))
        points.append(int(c[2]))

    graphs = [ctx.frame_graph(params, sils, bufs, masks=m) for m in masks]
    for k in range(args.warmup):
        graphs[k % len(graphs)].launch()
    torch.cuda.synchronize()

    K = args.steps
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        starts[k].record()
        graphs[k % len(graphs)].launch()
        ends[k].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    total_fine = sum(fine_vox[k % len(graphs)] for k in range(K))
    wall = t1 - t0
    value = total_fine / wall

    # dominant kernel: the persistent fine carve (with its one-workgroup job
    # builder), timed by the stage events of the eager runs
    fine_ms = float(np.mean(stage_ms["fine_carve"]))
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "fine voxels/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "frames": args.frames, "cameras": N,
                   "image": [W, H], "coarse_dims": list(sc0.coarse_dims), "fine_mm": sc0.hf_um / 1000,
                   "rois_per_frame_mean": float(np.mean(rois)),
                   "fine_voxels_per_frame_mean": float(np.mean(fine_vox)),
                   "surface_points_per_frame_mean": float(np.mean(points)),
                   "fine_tile": [tx, 256 // tx, tz]},
        "latency_ms": {"p50": pct(lat_ms, 50), "p99": pct(lat_ms, 99), "mean": float(np.mean(lat_ms))},
        "stages_ms": {s: float(np.mean(v)) for s, v in stage_ms.items()},
        "fine_carve_voxels_per_s": float(np.mean(fine_vox)) / (fine_ms * 1e-3),
    }

    tests = {}
    if not args.no_cpu_baseline:
        result["cpu_baseline"], tests = cpu_baseline(frames, args.cpu_seconds)

    # roofline of the dominant kernel: per fine voxel 1 B of occupancy written
    # plus one 4-byte silhouette word per (voxel, camera) test of the
    # index-order early exit (T, counted by the CPU baseline's run on the
    # same frames)
    if tests:
        vox = sum(tests[f][0] for f in tests)
        T = sum(tests[f][1] for f in tests)
        fine_ms_f = float(np.mean([stage_ms["fine_carve"][i] for i in range(len(stage_ms["fine_carve"]))
                                   if (i // max(1, args.stage_reps - 1)) in tests]))
        bytes_per_launch = (vox + 4 * T) / len(tests)
        achieved = bytes_per_launch / (fine_ms_f * 1e-3) / 1e9
        result["roofline"] = {"kernel": "fine carve (carve_persistent + frame_jobs)",
                              "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                              "bytes_per_launch": bytes_per_launch,
                              "tests_per_voxel": T / vox}
    print(json.dumps(result))


if __name__ == "__main__":
    main()
