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
lattice sizes over the timed frames / wall time of the timed loop), with
--in-flight frames overlapping (each on its own context, buffers and stream,
as a serving loop would run them; the figure for one frame at a time is
reported beside it), plus per-frame latency p50/p99 from HIP events around
each frame run one at a time.

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
# VALU ceiling of the exact test: 256 CUs x 4 SIMDs x 16 fp32 lanes x 2.4 GHz
# of non-packed issue (packed fp32 is not used), and the issue slots of one
# (sample, camera) test in this library's gfx950 code: 45 VALU instructions,
# one of them a quarter-rate v_rcp_f32 (48 slots).
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9
VALU_SLOTS_PER_TEST = 48


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed frames (the paper averages 200)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--frames", type=int, default=8, help="distinct synthetic frames cycled")
    ap.add_argument("--stage-reps", type=int, default=20, help="eager runs per frame for the stage split")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU-baseline time budget")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds-one-core", type=float, default=6.0,
                    help="budget of the oracle timed on one host thread (0 skips it)")
    ap.add_argument("--no-gather", action="store_true", help="skip the gather-ceiling leg")
    ap.add_argument("--no-judo", action="store_true", help="skip the judo-frame leg")
    ap.add_argument("--no-tiny", action="store_true", help="skip the tiny-rig leg")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the paper-shaped volleyball and the 2 mm judo legs")
    ap.add_argument("--judo-frames", type=int, default=2, help="distinct judo frames cycled")
    ap.add_argument("--judo-steps", type=int, default=50, help="timed judo frames")
    ap.add_argument("--no-h2d", action="store_true",
                    help="skip the frame latency that includes the silhouettes' host copy")
    ap.add_argument("--fine-tile", default="64x4", help="TXxTZ of the fine carve")
    ap.add_argument("--coarse-tile", default="64x1",
                    help="TXxTZ of the coarse carve (depth 4 culls cameras per tile, which at "
                         "coarse spacings costs more than it saves)")
    ap.add_argument("--in-flight", type=int, default=4,
                    help="frames in flight for the throughput figure (one context, buffer set "
                         "and stream each, one per hardware queue of the process: 4; measured "
                         "2, 4, 6, 8, 12: 2.5, 4.8, 4.5, 4.8, 4.7e10 fine voxels/s); latency is "
                         "measured one frame at a time")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-carve leg")
    ap.add_argument("--no-soft", action="store_true", help="skip the soft-hull leg")
    ap.add_argument("--no-mesh", action="store_true", help="skip the marching-cubes leg")
    ap.add_argument("--no-isovalue", action="store_true",
                    help="skip the Bresenham-isovalue leg")
    ap.add_argument("--no-visibility", action="store_true",
                    help="skip the depth-image and visibility leg")
    ap.add_argument("--batched-reps", type=int, default=10, help="timed batched-carve launches")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB before timing (a known-size "
                         "reference for hardware byte counters)")
    return ap.parse_args()


# Kernels whose roofline the bench reports: the stage that brackets each, its
# source files (a stored counter measurement is used only while they are
# unchanged) and the stored measurement.
KERNELS = {
    "fine_carve": {"kernel": "carve_frame_kernel", "stage": "fine_carve",
                   "sources": ["paper_1903_11785_amd/csrc/carve.hip",
                               "paper_1903_11785_amd/csrc/fvv_internal.h"],
                   "traffic": "profiles/carve_frame_kernel_volleyball_traffic.json"},
    "exit_points": {"kernel": "bisect_kernel", "stage": "exit_points",
                    "sources": ["paper_1903_11785_amd/csrc/surface.hip",
                                "paper_1903_11785_amd/csrc/fvv_internal.h"],
                    "traffic": "profiles/bisect_kernel_volleyball_traffic.json"},
}


def sources_sha256(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


BATCHED_KERNEL = {"kernel": "carve_batched_culled_kernel",
                  "sources": ["paper_1903_11785_amd/csrc/carve.hip",
                              "paper_1903_11785_amd/csrc/fvv_internal.h"],
                  "traffic": "profiles/carve_batched_culled_kernel_batched_traffic.json",
                  "tile": [16, 16, 4]}


VIS_KERNELS = {"kernel": "depth_clear_kernel + depth_raster_kernel + visibility_kernel",
               "sources": ["paper_1903_11785_amd/csrc/visibility.hip",
                           "paper_1903_11785_amd/csrc/fvv_internal.h"],
               "traffic": "profiles/visibility_volleyball_traffic.json"}


def stored_traffic(k):
    """HBM bytes per launch from the stored counter runs, if the kernel's sources
    are those the counters were taken on; else None."""
    spec = KERNELS[k] if isinstance(k, str) else k
    path = os.path.join(ROOT, spec["traffic"])
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != sources_sha256(spec["sources"]):
        return None
    return rec.get("traffic_bytes_per_launch")


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, np.float64), q))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_one_core(frames, budget_s):
    """The oracle on one host thread, on the same frames, until the budget is spent."""
    import oracle
    prev = oracle.set_threads(1)
    try:
        done_vox, spent, n = 0, 0.0, 0
        while spent < budget_s and n < 200:
            sc = frames[n % len(frames)]
            t0 = time.perf_counter()
            r = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims,
                             sc.t_np, sc.t_nb, sc.n_steps)
            spent += time.perf_counter() - t0
            done_vox += r.fine_voxels
            n += 1
        cores = oracle.threads()
    finally:
        oracle.set_threads(prev)
    return {"value": done_vox / spent, "unit": "fine voxels/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{n} whole volleyball-like frames on one host thread, {spent:.1f} s"}


def gather_leg(ctx, torch, sils, fine_vox, carve_ms, tests):
    """The gather ceiling of the fine carve: BW_g, the rate at which the GPU
    serves 4-byte words from a table the size of the frame's packed
    silhouettes (coalesced within a wave, random wave offsets, all CUs), and
    R_g = BW_g / (1 B + 4 B x mean tests per voxel) fine voxels/s; beside it
    the VALU ceiling of testing every voxel in camera order with the exact
    test, R_valu = VALU lane rate / (issue slots per test x mean tests per
    voxel).  achieved = fine voxels per frame / fine-carve kernel time."""
    table = sils.reshape(-1)
    ctx.gather_peak(table, reps=2)
    words = max(ctx.gather_peak(table, reps=20) for _ in range(3))
    bw = 4.0 * words
    # BW_hbm: a plain 1 GiB device-to-device copy (read + write bytes over its time)
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    bw_hbm = 10 * 2 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3)
    del a, b
    out = {"table_bytes": int(table.numel()) * 4, "bw_g_GBs": bw / 1e9,
           "bw_hbm_GBs": bw_hbm / 1e9,
           "kernel": "gather_peak_kernel (one coalesced 256 B wave read per step, global loads)"}
    if tests:
        t_mean = float(np.mean([tests[f]["tests_fine"] / tests[f]["vox"] for f in tests]))
        vox = float(np.mean([fine_vox[f] for f in tests]))
        ms = float(np.mean([carve_ms[f] for f in tests]))
        r_g = bw / (1.0 + 4.0 * t_mean)
        r_valu = VALU_LANE_PEAK / (VALU_SLOTS_PER_TEST * t_mean)
        achieved = vox / (ms * 1e-3)
        out.update({"tests_per_voxel": t_mean, "r_g_voxels_per_s": r_g,
                    "r_valu_voxels_per_s": r_valu, "achieved_voxels_per_s": achieved,
                    "frac": achieved / r_g, "frac_binding": achieved / min(r_g, r_valu),
                    "binding": "valu" if r_valu < r_g else "gather"})
    return out


def h2d_leg(args, fvv, torch, ctx, params, masks, sils, coarse, max_rois, max_fine, max_points,
            fine_vox):
    """Frame latency including the host-to-device copy of the packed
    silhouettes: each frame's packed words sit in pinned host memory; a step is
    the copy into the device buffer then the frame graph without the packing
    step, between HIP events on one stream, one frame at a time (as the frame
    latency without the copy is taken)."""
    host = []
    bufs = fvv.FrameBuffers(coarse, max_rois, max_fine, max_points)
    for m in masks:
        ctx.frame(params, sils, bufs, masks=m)
        torch.cuda.synchronize()
        h = torch.empty(sils.shape, dtype=sils.dtype, pin_memory=True)
        h.copy_(sils)
        host.append(h)
    g = ctx.frame_graph(params, sils, bufs)
    st = torch.cuda.Stream()
    K = min(args.steps, 200)
    for k in range(min(args.warmup, 10)):
        with torch.cuda.stream(st):
            sils.copy_(host[k % len(host)], non_blocking=True)
        g.launch(st)
    torch.cuda.synchronize()
    e0 = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    e1 = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    for k in range(K):
        with torch.cuda.stream(st):
            e0[k].record(st)
            sils.copy_(host[k % len(host)], non_blocking=True)
        g.launch(st)
        e1[k].record(st)
        st.synchronize()
        if k < len(host) and int(bufs.counts[1].item()) != fine_vox[k]:
            raise RuntimeError("frame from host-copied silhouettes differs")
    lat = [a.elapsed_time(b) for a, b in zip(e0, e1)][len(host):]
    return {"latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "mean": float(np.mean(lat)),
                           "max": float(np.max(lat))},
            "copied_bytes": int(sils.numel()) * 4, "frames": len(lat),
            "note": "packed silhouettes copied from pinned host memory, then the frame graph"}


JUDO_WORKLOAD = ("judo-like frame: 24 cams 3840x2160, 1-2 touching pairs, 10x10x3 m mat, "
                 "coarse 40 mm, fine 5 mm")


TINY_WORKLOAD = ("tiny rig: 4 cams 320x240, 2 ellipsoids, 4x4x2 m, coarse 62.5 mm (64x64x32), fine 20 mm; "
                 "seeds 0-7, one frame each")

PAPER_V_WORKLOAD = ("the paper's volleyball shape: 10 cams 3840x2160 (f ~3000 px), 14 players, "
                    "18x18x9 m, coarse 50 mm (360x360x180), fine 20 mm")

JUDO_FINE_WORKLOAD = ("judo-like frame at 2 mm: 24 cams 3840x2160, 10x10x3 m, coarse 40 mm, "
                      "fine 2 mm (~1.9e8 fine samples in 6 ROIs)")


def config_leg(args, fvv, torch, cpu, cfg, n_frames, steps, workload, cpu_frames,
               max_fine=1 << 27, stage_reps=0):
    """Another configuration through the whole path: its frames one at a time
    as a HIP graph between HIP events (latency p50/p99 and fine voxels carved
    per second of frame time), with the oracle timed on its first cpu_frames
    frames on all host threads; with stage_reps, also the per-stage split and
    the two big kernels' own times from eager runs with the frame's events."""
    import scenes
    frames = [scenes.make_scene(cfg, f) for f in range(max(1, n_frames))]
    sc0 = frames[0]
    N, H, W = sc0.masks.shape
    coarse = fvv.Grid(origin=tuple(sc0.origin), h=sc0.hc, lo=(0, 0, 0), dims=sc0.coarse_dims)
    max_rois, max_points = 256, 1 << 23
    ctx = fvv.Context(max_cams=N, max_w=W, max_h=H, max_coarse=coarse.size, max_fine=max_fine,
                      max_rois=max_rois, max_points=max_points, max_jobs=max_rois)
    try:
        tx, tz = (int(v) for v in args.fine_tile.split("x"))
        ctx_, ctz = (int(v) for v in args.coarse_tile.split("x"))
        params = fvv.frame_params(sc0.P32, W, H, coarse, sc0.hc_um, sc0.hf_um, sc0.t_np,
                                  sc0.t_nb, sc0.n_steps, coarse_tile=fvv.tile(ctx_, ctz),
                                  fine_tile=fvv.tile(tx, tz))
        masks = [torch.from_numpy(sc.masks).cuda() for sc in frames]
        sils = torch.empty((N, H, (W + 31) // 32), dtype=torch.int32, device="cuda")
        bufs = fvv.FrameBuffers(coarse, max_rois, max_fine, max_points)
        fine, rois, points = [], [], []
        for m in masks:
            ctx.frame(params, sils, bufs, masks=m)
            torch.cuda.synchronize()
            if ctx.check() != fvv.FVV_OK:
                raise RuntimeError("frame exceeded a capacity")
            c = bufs.counts.cpu().numpy()
            rois.append(int(c[0]))
            fine.append(int(c[1]))
            points.append(int(c[2]))
        graphs = [ctx.frame_graph(params, sils, bufs, masks=m) for m in masks]
        for k in range(5):
            graphs[k % len(graphs)].launch()
        torch.cuda.synchronize()
        K = max(1, steps)
        e0 = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
        e1 = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
        for k in range(K):
            e0[k].record()
            graphs[k % len(graphs)].launch()
            e1[k].record()
        torch.cuda.synchronize()
        lat = [a.elapsed_time(b) for a, b in zip(e0, e1)]
        done = sum(fine[k % len(graphs)] for k in range(K))
        out = {"workload": workload, "frames": len(frames), "steps": K,
               "rois_per_frame_mean": float(np.mean(rois)),
               "fine_voxels_per_frame_mean": float(np.mean(fine)),
               "surface_points_per_frame_mean": float(np.mean(points)),
               "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99),
                              "mean": float(np.mean(lat))},
               "fine_voxels_per_s_one_frame_at_a_time": done / (sum(lat) * 1e-3)}
        for g in graphs:
            g.close()
        if stage_reps > 0:
            st = {k: [] for k in fvv.STAGES}
            kt = {k: [] for k in fvv.FRAME_KERNELS}
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(fvv.FRAME_EVENTS)]
            for rep in range(stage_reps + 1):
                for m in masks:
                    ctx.frame(params, sils, bufs, masks=m, events=ev)
                    torch.cuda.synchronize()
                    if rep == 0:
                        continue
                    for i, k in enumerate(fvv.STAGES):
                        st[k].append(ev[i].elapsed_time(ev[i + 1]))
                    for q, k in enumerate(fvv.FRAME_KERNELS):
                        kt[k].append(ev[fvv.FRAME_STAGE_EVENTS + 2 * q].elapsed_time(
                            ev[fvv.FRAME_STAGE_EVENTS + 2 * q + 1]))
            out["stages_ms"] = {k: float(np.mean(v)) for k, v in st.items()}
            out["kernels_ms"] = {k: float(np.mean(v)) for k, v in kt.items()}
        del graphs, bufs, masks, sils
    finally:
        torch.cuda.synchronize()
        ctx.close()
    if cpu:
        import oracle
        n_cpu = min(len(frames), max(1, cpu_frames))
        done, t = 0, 0.0
        for f in range(n_cpu):
            sc = frames[f]
            t0 = time.perf_counter()
            r = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims,
                             sc.t_np, sc.t_nb, sc.n_steps)
            t += time.perf_counter() - t0
            if r.fine_voxels != fine[f]:
                raise RuntimeError("oracle and GPU fine voxel counts differ")
            done += r.fine_voxels
        out["cpu_baseline"] = {"value": done / t, "unit": "fine voxels/s",
                               "cores": oracle.threads(), "kind": "oracle",
                               "sample": f"{n_cpu} frame(s) of this configuration, {t:.2f} s"}
    return out


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
        tests[n % len(frames)] = {"vox": r.fine_voxels, "tests_fine": r.tests_fine,
                                  "edges": int(sum(k.size for k in r.keys)),
                                  "tests_surface": r.tests_surface}
        n += 1
    return {"value": done_vox / spent, "unit": "fine voxels/s", "cores": oracle.threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{n} whole volleyball-like frames (same inputs as the GPU steps), "
                      f"{spent:.1f} s of oracle time on host CPU"}, tests


BATCHED_WORKLOAD = ("batched fine carve: 64 frames of the tiny rig (4 cams 320x240) x 12 ROI boxes "
                    "with edges U[0.6, 2.5] m at 10 mm")


def batched_leg(args, fvv, torch):
    """The batched workload: one persistent launch (captured as a HIP graph)
    carving 64 frames x 12 uneven ROIs with the autotuned tile, against the
    same ROIs as 768 fvv_carve launches (captured as one graph too, so launch
    gaps count but host overhead does not); the outputs must be identical."""
    import scenes
    from paper_1903_11785_amd import autotune
    scs, boxes = scenes.batched_rois()
    N = scs[0].P32.shape[0]
    W, H = scs[0].W, scs[0].H
    ctx = fvv.Context(max_cams=N, max_w=W, max_h=H, max_coarse=1, max_fine=1, max_rois=1,
                      max_points=1, max_jobs=len(boxes))
    P_all = np.concatenate([s.P32 for s in scs], 0)
    sils = ctx.pack_silhouettes(torch.from_numpy(np.concatenate([s.masks for s in scs], 0)).cuda())
    cams_dev = fvv.cameras_to_device(P_all, W, H)
    jobs, total = fvv.frame_major_jobs([(b.frame, b.lo, b.dims) for b in boxes],
                                       [s.origin for s in scs], [s.hf for s in scs], N, W, H)
    jobs_d = fvv.jobs_to_device(jobs)
    out = torch.empty(total, dtype=torch.uint8, device="cuda")
    tuned = autotune.tune_batched(ctx, jobs, jobs_d, cams_dev, P_all, sils, out, reps=2)
    t = tuned["tile"]
    g = ctx.carve_batched_graph(jobs_d, len(boxes), cams_dev, sils, out, t)
    for _ in range(2):
        g.launch()
    torch.cuda.synchronize()
    ms = []
    for _ in range(max(1, args.batched_reps)):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.launch()
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    if ctx.check() != fvv.FVV_OK:
        raise RuntimeError("batched carve reported an invalid job")

    # the same ROIs, one fvv_carve launch each
    per = torch.empty(total, dtype=torch.uint8, device="cuda")
    grids = [fvv.Grid(origin=tuple(np.float32(scs[b.frame].origin)), h=np.float32(scs[b.frame].hf),
                      lo=tuple(b.lo), dims=tuple(b.dims)) for b in boxes]
    offs = [int(j["out_offset"]) for j in jobs]

    def per_roi(stream=None):
        for b, gr, o in zip(boxes, grids, offs):
            ctx.carve(scs[b.frame].P32, W, H, sils[b.frame * N:(b.frame + 1) * N], gr,
                      out=per[o:o + gr.size], stream=stream)

    per_roi()                                     # eager, once (also the warm-up)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per_roi()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3
    pg = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(pg, stream=side):
            per_roi(stream=side)
    torch.cuda.current_stream().wait_stream(side)
    per_ms = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        pg.replay()
        e1.record()
        e1.synchronize()
        per_ms.append(e0.elapsed_time(e1))
    identical = bool(torch.equal(out, per))
    del pg, per
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on the ROIs of the first 4 frames, all host threads; its
        # occupancies must equal the batched launch's bytes
        import oracle
        sel = [q for q, b in enumerate(boxes) if b.frame < 4]
        host_sils = {f: oracle.pack(scs[f].masks) for f in range(4)}
        done, spent = 0, 0.0
        for q in sel:
            b = boxes[q]
            lat = oracle.Lattice(origin=np.asarray(scs[b.frame].origin, np.float32),
                                 h=np.float32(scs[b.frame].hf), lo=tuple(b.lo), dims=tuple(b.dims))
            t0 = time.perf_counter()
            ref, _ = oracle.carve(scs[b.frame].P32, host_sils[b.frame], W, H, lat)
            spent += time.perf_counter() - t0
            o = offs[q]
            got = out[o:o + lat.size].cpu().numpy()
            if not np.array_equal(got, ref.reshape(-1)):
                raise RuntimeError("batched carve differs from the oracle")
            done += lat.size
        cpu = {"value": done / spent, "unit": "samples/s", "cores": oracle.threads(),
               "kind": "oracle",
               "sample": f"the {len(sel)} ROIs of the first 4 frames ({done} samples), {spent:.2f} s"}
    ctx.close()
    b_ms, p_ms = pct(ms, 50), pct(per_ms, 50)
    achieved = total / (b_ms * 1e-3) / 1e9
    return {
        "cpu_baseline": cpu,
        "workload": BATCHED_WORKLOAD, "rois": len(boxes), "samples": int(total),
        "tile": [t.tx, t.ty, t.tz, t.persistent_blocks], "tuner_key": tuned["key"],
        "tuner_ms": {f"{tx}x{256 // tx}x{tz}/{blk}": round(m, 4)
                     for (tx, tz, blk, m) in tuned["table"]},
        "batch_ms_p50": b_ms, "batch_ms_min": float(min(ms)), "per_frame_ms": b_ms / 64,
        "samples_per_s": total / (b_ms * 1e-3),
        "per_roi_graph_ms_p50": p_ms, "per_roi_eager_wall_ms": eager_ms,
        "speedup_vs_per_roi": p_ms / b_ms, "identical_to_per_roi": identical,
        # compulsory bytes only: one occupancy byte per sample written; traffic from
        # the stored counter runs (taken with the 16x16x4 tile)
        "roofline": {"kernel": "carve_batched_culled_kernel", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": int(total),
                     "traffic": (stored_traffic(BATCHED_KERNEL)
                                 if [t.tx, t.ty, t.tz] == BATCHED_KERNEL["tile"] else None)},
    }


SOFT_WORKLOAD = ("soft hull: 16 cams 320x240 on the tiny ring, poses perturbed 0.5 deg / 1 cm, "
                 "fp32 logits, the 2 cm lattice around one object, L2 loss to its occupancy")


def soft_leg(args, fvv, torch):
    """The differentiable soft hull: forward (fused L2 loss) and forward plus
    adjoint (logit and pose gradients) through the autograd function."""
    import scenes
    from paper_1903_11785_amd.soft import SoftHull
    s = scenes.scene_soft(0)
    K, R0, t0 = s.base_pose()
    N = K.shape[0]
    ctx = fvv.Context(max_cams=N, max_w=s.W, max_h=s.H, max_coarse=1, max_fine=1, max_rois=1,
                      max_points=1, max_jobs=1)
    grid = fvv.Grid(origin=tuple(np.float32(s.origin)), h=np.float32(s.h), lo=s.lo, dims=s.dims)
    hull = SoftHull(ctx, grid, K, R0, t0, s.W, s.H)
    L = torch.from_numpy(s.logits).cuda().requires_grad_(True)
    w = torch.from_numpy(s.omega).requires_grad_(True)
    t = torch.from_numpy(s.tau).requires_grad_(True)
    target = torch.from_numpy(s.target.reshape(-1)).cuda()

    def step(backward):
        if backward:
            loss = hull.l2_loss(L, w, t, target)
            return torch.autograd.grad(loss, (L, w, t))
        with torch.no_grad():
            return hull.l2_loss(L, w, t, target)

    reps = 20
    out = {}
    for name, bw in (("forward_ms", False), ("forward_backward_ms", True)):
        for _ in range(3):
            step(bw)
        torch.cuda.synchronize()
        t0_ = time.perf_counter()
        for _ in range(reps):
            step(bw)
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0_) * 1e3 / reps
    V = int(np.prod(s.dims))
    # the library's forward (fused L2 loss) and adjoint calls alone: ten calls
    # captured in a graph, replayed between events, per call
    cams = hull.cameras(w, t)
    Ld = L.detach()
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    gl = torch.empty_like(Ld)
    gp = torch.empty((N, 6), dtype=torch.float64, device="cuda")
    scale = torch.ones(1, dtype=torch.float64, device="cuda")

    def fwd(stream=None):
        for _ in range(10):
            ctx.soft_forward(grid, cams, s.W, s.H, Ld, target=target, loss=loss, stream=stream)

    def bwd(stream=None):
        for _ in range(10):
            ctx.soft_backward(grid, cams, s.W, s.H, Ld, gl, gp, target=target, scale=scale,
                              stream=stream)

    f_ms = pct(graph_ms(torch, fwd, 11), 50) / 10
    b_ms = pct(graph_ms(torch, bwd, 11), 50) / 10
    ctx.close()
    # algorithmic bytes: forward, per sample 4 B of target read and per (sample,
    # camera) the four bilinear taps' 4 B logits; adjoint, per sample 4 B of
    # target and per (sample, camera) the four taps read and four 4 B logit
    # gradients added (the pose sums are per camera)
    f_bytes = V * (4 + 16 * N)
    b_bytes = V * (4 + 32 * N)
    rl = {}
    for name, ms, by, kern in (("forward", f_ms, f_bytes, "soft_fwd_kernel"),
                               ("backward", b_ms, b_bytes, "soft_bwd_kernel + soft_pose_kernel")):
        achieved = by / (ms * 1e-3) / 1e9
        rl[name] = {"kernel": kern, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "bytes_per_call": int(by), "call_ms": ms}
    return {"workload": SOFT_WORKLOAD, "samples": V, "cameras": N,
            "forward_ms": out["forward_ms"], "forward_backward_ms": out["forward_backward_ms"],
            "samples_per_s_forward_backward": V / (out["forward_backward_ms"] * 1e-3),
            "note": "wall time per call through the autograd function, including the host-side "
                    "pose set-up and the copy of the pose gradients to the host",
            "kernel_call_ms": {"forward": f_ms, "backward": b_ms},
            "roofline": rl["backward"], "rooflines": rl}


def graph_ms(torch, enqueue, reps):
    """GPU time of the calls enqueue(stream) makes, captured once as a graph
    on a side stream (so host-side marshalling is not timed) and replayed reps
    times between HIP events; the first replay is a warm-up."""
    enqueue()                                    # eager once (warm-up, lazy set-up)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            enqueue(side)
    torch.cuda.current_stream().wait_stream(side)
    out = []
    for r in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        e1.synchronize()
        if r > 0:
            out.append(e0.elapsed_time(e1))
    del g
    return out


def mesh_leg(args, fvv, torch, ctx, params, masks, sils, coarse, max_rois, max_fine, max_points,
             lat_no_mesh_ms):
    """Marching-cubes triangles of the volleyball frames: (1) the frame graph
    with its mesh branch (triangle count beside the crossing edges, triangles
    beside the exit points, on the side stream), one frame at a time, against
    the same frames without it; (2) fvv_mesh on each ROI of one frame (fine
    occupancy and keys as the frame left them), timed with HIP events on its
    stream: bitmap, word edges, count and write passes."""
    max_tris = 1 << 23
    bufs = fvv.FrameBuffers(coarse, max_rois, max_fine, max_points, max_tris=max_tris)
    graphs = [ctx.frame_graph(params, sils, bufs, masks=m) for m in masks]
    n_tris = []
    for g in graphs:
        g.launch()
        torch.cuda.synchronize()
        K = int(bufs.counts.cpu()[0])
        n_tris.append(int(bufs.tri_off[K].cpu()))
    if ctx.check() != fvv.FVV_OK:
        raise RuntimeError("mesh exceeded a capacity")
    steps = max(1, min(args.steps, 100))
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for k in range(steps):
        ev[k][0].record()
        graphs[k % len(graphs)].launch()
        ev[k][1].record()
    torch.cuda.synchronize()
    lat = [a.elapsed_time(b) for a, b in ev]
    for g in graphs:
        g.close()

    # fvv_mesh, ROI by ROI, on frame 0's outputs
    graphs0 = ctx.frame_graph(params, sils, bufs, masks=masks[0])
    graphs0.launch()
    torch.cuda.synchronize()
    graphs0.close()
    K = int(bufs.counts.cpu()[0])
    jobs = bufs.jobs_host(K)
    poff = bufs.point_off.cpu().numpy().view(np.uint32)
    tris = torch.empty((max_tris, 3), dtype=torch.int32, device="cuda")
    n_t = torch.zeros(1, dtype=torch.int32, device="cuda")
    calls = []
    for t in range(K):
        g = jobs[t]
        dims = tuple(int(v) for v in g["dims"])
        grid = fvv.Grid(origin=tuple(g["origin"]), h=g["h"], lo=tuple(int(v) for v in g["lo"]),
                        dims=dims)
        o = int(g["out_offset"])
        occ = bufs.occ_fine[o:o + int(np.prod(dims))]
        keys = bufs.keys[int(poff[t]):int(poff[t + 1])]
        nk = torch.tensor([int(poff[t + 1] - poff[t])], dtype=torch.int32, device="cuda")
        calls.append((grid, occ, keys, nk))
    bytes_total = 0
    for grid, occ, keys, nk in calls:
        ctx.mesh(grid, occ, keys, nk, tris=tris, n_tris=n_t)
        bytes_total += grid.size + 4 * keys.numel() + 12 * int(n_t.cpu()[0])

    def all_rois(stream=None):
        for grid, occ, keys, nk in calls:
            ctx.mesh(grid, occ, keys, nk, tris=tris, n_tris=n_t, stream=stream)

    per_call = graph_ms(torch, all_rois, reps=6)
    if ctx.check() != fvv.FVV_OK:
        raise RuntimeError("fvv_mesh reported a missing vertex")
    frame_ms = pct(per_call, 50)
    achieved = bytes_total / (frame_ms * 1e-3) / 1e9
    return {
        "workload": "marching-cubes triangles of the volleyball frames' ROIs",
        "triangles_per_frame_mean": float(np.mean(n_tris)),
        "frame_latency_ms_with_mesh": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "frame_latency_ms_without_mesh_p50": lat_no_mesh_ms,
        "mesh_branch_added_ms_p50": pct(lat, 50) - lat_no_mesh_ms,
        "fvv_mesh_per_roi": {"rois": K, "ms_per_frame_p50": frame_ms,
                             "ms_per_roi": frame_ms / max(K, 1),
                             "roofline": {"bound": "hbm", "achieved": achieved,
                                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                          "frac": achieved / HBM_PEAK_GBS,
                                          "bytes_per_frame": bytes_total,
                                          "traffic": None,
                                          "note": "compulsory bytes: 1 B occupancy per sample read, "
                                                  "4 B per key read, 12 B per triangle written; "
                                                  "six launches per ROI, the frame's calls "
                                                  "captured as one graph"}},
    }


def isovalue_leg(args, fvv, torch, ctx, params, masks, sils, coarse, max_rois, max_fine,
                 max_points, frame0, exit_points_ms):
    """The paper's Bresenham isovalue (fvv_isovalue) on every ROI of one
    volleyball frame, on the frame's own fine occupancy and keys, timed with
    HIP events around each call, beside the frame's exit-point bisection; and
    how far lambda lies from the bisection's t* on the same edges."""
    bufs = fvv.FrameBuffers(coarse, max_rois, max_fine, max_points)
    g = ctx.frame_graph(params, sils, bufs, masks=masks[0])
    g.launch()
    torch.cuda.synchronize()
    g.close()
    K = int(bufs.counts.cpu()[0])
    jobs = bufs.jobs_host(K)
    poff = bufs.point_off.cpu().numpy().view(np.uint32)
    N = frame0.P32.shape[0]
    calls = []
    for t in range(K):
        j = jobs[t]
        dims = tuple(int(v) for v in j["dims"])
        grid = fvv.Grid(origin=tuple(j["origin"]), h=j["h"], lo=tuple(int(v) for v in j["lo"]),
                        dims=dims)
        o = int(j["out_offset"])
        keys = bufs.keys[int(poff[t]):int(poff[t + 1])]
        nk = torch.tensor([keys.numel()], dtype=torch.int32, device="cuda")
        lam = torch.empty(keys.numel(), dtype=torch.float32, device="cuda")
        xyz = torch.empty((keys.numel(), 3), dtype=torch.float32, device="cuda")
        calls.append((grid, bufs.occ_fine[o:o + int(np.prod(dims))], keys, nk, lam, xyz))
    def all_rois(stream=None):
        for grid, occ, keys, nk, lam, xyz in calls:
            ctx.isovalue(grid, occ, frame0.P32, frame0.W, frame0.H, sils, keys, nk, lam=lam,
                         xyz=xyz, stream=stream)

    per_frame = graph_ms(torch, all_rois, reps=6)
    # lambda against t* (the bisection's bracket midpoint, from its point)
    E = int(poff[K])
    keys_h = bufs.keys[:E].cpu().numpy().view(np.uint32)
    xyz_h = bufs.xyz[:E].cpu().numpy()
    lam_h = np.concatenate([c[4].cpu().numpy() for c in calls])
    diffs = []
    for t in range(K):
        j = jobs[t]
        a, b = int(poff[t]), int(poff[t + 1])
        k = keys_h[a:b]
        nx, ny = int(j["dims"][0]), int(j["dims"][1])
        lin, axis = k // 3, k % 3
        gi = np.stack([lin % nx, (lin // nx) % ny, lin // (nx * ny)], 1) + np.asarray(j["lo"])
        occ = calls[t][1].cpu().numpy()
        on_first = occ[lin] != 0
        g_on = gi[np.arange(k.size), axis] + np.where(on_first, 0, 1)
        x_on = np.asarray(j["origin"], np.float64)[axis] + g_on * float(j["h"])
        tstar = np.abs(xyz_h[a:b][np.arange(k.size), axis] - x_on) / float(j["h"])
        diffs.append(lam_h[a:b] - tstar)
    d = np.concatenate(diffs) if diffs else np.zeros(1)
    # the whole frame with the Bresenham estimator in place of the bisection
    pb = fvv.frame_params(frame0.P32, frame0.W, frame0.H, coarse, frame0.hc_um, frame0.hf_um,
                          frame0.t_np, frame0.t_nb, frame0.n_steps,
                          coarse_tile=params.coarse_tile, fine_tile=params.fine_tile,
                          exit_estimator=fvv.EXIT_BRESENHAM)
    gb = [ctx.frame_graph(pb, sils, bufs, masks=m) for m in masks]
    for gg in gb:
        gg.launch()
    torch.cuda.synchronize()
    if ctx.check() != fvv.FVV_OK:
        raise RuntimeError("frame with the Bresenham estimator exceeded a capacity")
    lat_b = []
    for k in range(max(1, min(args.steps, 100))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gb[k % len(gb)].launch()
        e1.record()
        e1.synchronize()
        lat_b.append(e0.elapsed_time(e1))
    for gg in gb:
        gg.close()
    ms = pct(per_frame, 50)
    bytes_per_frame = E * (4 + 1 + 16) + E * N * 8
    achieved = bytes_per_frame / (ms * 1e-3) / 1e9
    return {
        "workload": "Bresenham isovalue (Eq. (2)-(3)) of one volleyball frame's crossing edges",
        "edges": E, "rois": K, "ms_per_frame_p50": ms, "edges_per_s": E / (ms * 1e-3),
        "exit_points_bisection_stage_ms": exit_points_ms,
        "frame_latency_ms_bresenham_estimator": {"p50": pct(lat_b, 50), "p99": pct(lat_b, 99)},
        "lambda_minus_tstar": {"mean": float(d.mean()), "mean_abs": float(np.abs(d).mean()),
                               "p90_abs": float(np.percentile(np.abs(d), 90))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "bytes_per_frame": int(bytes_per_frame),
                     "traffic": None,
                     "note": "per edge 4 B key + 1 B occupancy + 16 B out, per (edge, camera) "
                             "two 4 B silhouette words (start and one step); one launch per ROI, "
                             "the frame's calls captured as one graph"},
    }


def visibility_leg(args, fvv, torch, ctx, params, masks, sils, coarse, max_rois, max_fine,
                   max_points, frame0, t_v=0.1):
    """Depth images and visibility (Sec. II-D) of one volleyball frame's mesh
    (the frame's exit points and marching-cubes triangles) in its cameras,
    the call captured as a graph and replayed between HIP events."""
    bufs = fvv.FrameBuffers(coarse, max_rois, max_fine, max_points, max_tris=1 << 22)
    g = ctx.frame_graph(params, sils, bufs, masks=masks[0])
    g.launch()
    torch.cuda.synchronize()
    g.close()
    K = int(bufs.counts.cpu()[0])
    n_t = bufs.tri_off[K:K + 1]
    n_p = bufs.counts[2:3]
    N = frame0.P32.shape[0]
    depth = torch.empty((N, frame0.H, frame0.W), dtype=torch.float32, device="cuda")
    vis = torch.empty(bufs.tris.shape[0], dtype=torch.int32, device="cuda")

    def call(stream=None):
        ctx.visibility(frame0.P32, frame0.W, frame0.H, bufs.xyz, n_p, bufs.tris, n_t, t_v,
                       depth=depth, vis=vis, stream=stream)

    ms_all = graph_ms(torch, call, reps=8)
    if ctx.check() != fvv.FVV_OK:
        raise RuntimeError("visibility leg reported an error")
    T = int(n_t.cpu()[0])
    covered = int(torch.isfinite(depth).sum())
    v = vis[:T].cpu().numpy().view(np.uint32)
    seen = np.unpackbits(v.view(np.uint8)).reshape(-1, 32).sum(1) if T else np.zeros(1)
    ms = pct(ms_all, 50)
    px = N * frame0.W * frame0.H
    bytes_ = 4 * px + 4 * covered + T * (12 + 36 + 4 + 4 * N)
    achieved = bytes_ / (ms * 1e-3) / 1e9
    return {
        "workload": "depth images (Eq. (4)) and visibility of one volleyball frame's mesh in its "
                    "16 cameras at 1920x1080, T_v = 0.1 m",
        "triangles": T, "cameras": N, "covered_pixels": covered,
        "ms_per_frame_p50": ms, "triangle_cameras_per_s": T * N / (ms * 1e-3),
        "cameras_seeing_a_triangle_mean": float(seen.mean()),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "bytes_per_frame": int(bytes_),
                     "traffic": stored_traffic(VIS_KERNELS),
                     "note": "4 B per depth pixel cleared, 4 B per covered pixel written, per "
                             "triangle 12 B indices + 36 B vertices + 4 B mask + 4 B of depth "
                             "per camera; three kernels"},
    }


def soft_cpu_baseline():
    """The soft-hull oracle (float64 PyTorch CPU: forward + autograd) on the
    same scene, timed once."""
    import scenes
    from oracle import soft as osoft
    s = scenes.scene_soft(0)
    K, R0, t0 = s.base_pose()
    t0_ = time.perf_counter()
    osoft.soft_grad(s.logits, K, R0, t0, s.omega, s.tau, s.origin, s.h, s.lo, s.dims,
                    target=s.target)
    import torch
    return {"forward_backward_ms": (time.perf_counter() - t0_) * 1e3, "kind": "oracle",
            "cores": torch.get_num_threads(), "sample": "one forward + gradient of the same scene"}


def progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this path runs on one GPU; more than one GPU is not supported. "
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
    ctx_, ctz = (int(v) for v in args.coarse_tile.split("x"))
    params = fvv.frame_params(sc0.P32, W, H, coarse, sc0.hc_um, sc0.hf_um, sc0.t_np, sc0.t_nb,
                              sc0.n_steps, coarse_tile=fvv.tile(ctx_, ctz),
                              fine_tile=fvv.tile(tx, tz))
    masks = [torch.from_numpy(sc.masks).cuda() for sc in frames]
    sils = torch.empty((N, H, (W + 31) // 32), dtype=torch.int32, device="cuda")
    bufs = fvv.FrameBuffers(coarse, max_rois, max_fine, max_points)

    # per-frame work (from one eager run each) and the per-stage split
    fine_vox, rois, points = [], [], []
    stage_ms = {s: [] for s in fvv.STAGES}
    stage_ms_frame = {s: [[] for _ in masks] for s in fvv.STAGES}
    # the kernels' own execution times (events that take the kernel's start and
    # end, on the stream the kernel runs on)
    kernel_ms_frame = {k: [[] for _ in masks] for k in fvv.FRAME_KERNELS}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(fvv.FRAME_EVENTS)]
    for f, m in enumerate(masks):
        for rep in range(max(1, args.stage_reps)):
            ctx.frame(params, sils, bufs, masks=m, events=ev)
            torch.cuda.synchronize()
            if rep > 0:
                for i, s in enumerate(fvv.STAGES):
                    dt = ev[i].elapsed_time(ev[i + 1])
                    stage_ms[s].append(dt)
                    stage_ms_frame[s][f].append(dt)
                for q, k in enumerate(fvv.FRAME_KERNELS):
                    e0 = ev[fvv.FRAME_STAGE_EVENTS + 2 * q]
                    kernel_ms_frame[k][f].append(e0.elapsed_time(ev[fvv.FRAME_STAGE_EVENTS + 2 * q + 1]))
        if ctx.check() != fvv.FVV_OK:
            raise RuntimeError("frame exceeded a capacity")
        c = bufs.counts.cpu().numpy()
        rois.append(int(c[0]))
        fine_vox.append(int(c[1]))
        points.append(int(c[2]))

    if args.calib_copy_mib > 0:              # known-size reference for byte counters
        a = torch.empty(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    progress("volleyball frames: stage split done, timing the frame graphs")
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
    wall_seq = t1 - t0

    # throughput with frames in flight: slot k % n_slots runs frame k on its own
    # context, buffers and stream (a slot's frames follow each other on its stream)
    n_slots = max(1, args.in_flight)
    slots = [(ctx, sils, bufs, graphs)]
    for _ in range(n_slots - 1):
        c2 = fvv.Context(max_cams=N, max_w=W, max_h=H, max_coarse=coarse.size, max_fine=max_fine,
                         max_rois=max_rois, max_points=max_points, max_jobs=max_rois)
        s2 = torch.empty_like(sils)
        b2 = fvv.FrameBuffers(coarse, max_rois, max_fine, max_points)
        slots.append((c2, s2, b2, [c2.frame_graph(params, s2, b2, masks=m) for m in masks]))
    streams = [torch.cuda.Stream() for _ in range(n_slots)]
    for k in range(args.warmup):
        slots[k % n_slots][3][k % len(masks)].launch(streams[k % n_slots])
    torch.cuda.synchronize()
    starts_p = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    ends_p = [torch.cuda.Event(enable_timing=True) for _ in range(K)]
    t0 = time.perf_counter()
    for k in range(K):
        st = streams[k % n_slots]
        starts_p[k].record(st)
        slots[k % n_slots][3][k % len(masks)].launch(st)
        ends_p[k].record(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat_p = [s.elapsed_time(e) for s, e in zip(starts_p, ends_p)]
    for c2, _, _, _ in slots[1:]:
        if c2.check() != fvv.FVV_OK:
            raise RuntimeError("frame exceeded a capacity")
    wall = t1 - t0
    value = total_fine / wall

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
                   "fine_tile": [tx, 256 // tx, tz], "coarse_tile": [ctx_, 256 // ctx_, ctz]},
        "in_flight": n_slots,
        "value_one_frame_at_a_time": total_fine / wall_seq,
        "latency_ms": {"p50": pct(lat_ms, 50), "p99": pct(lat_ms, 99), "mean": float(np.mean(lat_ms))},
        "latency_ms_in_flight": {"p50": pct(lat_p, 50), "p99": pct(lat_p, 99),
                                 "mean": float(np.mean(lat_p))},
        "stages_ms": {s: float(np.mean(v)) for s, v in stage_ms.items()},
    }

    if not args.no_mesh:
        progress("mesh leg")
        result["mesh"] = mesh_leg(args, fvv, torch, ctx, params, masks, sils, coarse, max_rois,
                                  max_fine, max_points, pct(lat_ms, 50))
    if not args.no_isovalue:
        progress("isovalue leg")
        result["isovalue"] = isovalue_leg(args, fvv, torch, ctx, params, masks, sils, coarse,
                                          max_rois, max_fine, max_points, sc0,
                                          float(np.mean(stage_ms_frame["exit_points"][0])))
    if not args.no_visibility:
        progress("visibility leg")
        result["visibility"] = visibility_leg(args, fvv, torch, ctx, params, masks, sils, coarse,
                                              max_rois, max_fine, max_points, sc0)
    if not args.no_batched:
        progress("batched leg")
        result["batched"] = batched_leg(args, fvv, torch)
    if not args.no_soft:
        progress("soft hull leg")
        result["soft_hull"] = soft_leg(args, fvv, torch)
        if not args.no_cpu_baseline:
            result["soft_hull"]["cpu_baseline"] = soft_cpu_baseline()

    if not args.no_judo:
        progress("judo leg")
        result["judo"] = config_leg(args, fvv, torch, not args.no_cpu_baseline, scenes.CFG_JUDO,
                                    args.judo_frames, args.judo_steps, JUDO_WORKLOAD, 1)
    if not args.no_tiny:
        progress("tiny leg")
        result["tiny"] = config_leg(args, fvv, torch, not args.no_cpu_baseline, scenes.CFG_TINY,
                                    8, 50, TINY_WORKLOAD, 8)
    if not args.no_paper:
        progress("paper-shaped volleyball and 2 mm judo legs")
        # the paper's own volleyball shape, with its Table II times (1st volleyball
        # sequence, steps B-1 to C, GTX 1080 Ti) beside it as context
        pv = config_leg(args, fvv, torch, not args.no_cpu_baseline, scenes.CFG_PAPER_V, 2, 50,
                        PAPER_V_WORKLOAD, 1, stage_reps=5)
        pv["paper_table_ii_ms"] = {"hardware": "GTX 1080 Ti", "sequence": "1st volleyball",
                                   "B1_sparse_hull": 0.54, "B2_noise_filter_roi": 21.49,
                                   "B3_dense_hull": 1.23, "C_polygonization": 3.90,
                                   "B1_to_C": 27.16}
        result["paper_volleyball"] = pv
        result["judo_fine"] = config_leg(args, fvv, torch, not args.no_cpu_baseline,
                                         scenes.CFG_JUDO_FINE, 1, 10, JUDO_FINE_WORKLOAD, 1,
                                         max_fine=1 << 28, stage_reps=3)
    if not args.no_h2d:
        progress("host-copy latency leg")
        result["latency_with_h2d"] = h2d_leg(args, fvv, torch, ctx, params, masks, sils, coarse,
                                             max_rois, max_fine, max_points, fine_vox)

    tests = {}
    if not args.no_cpu_baseline:
        progress("oracle baseline")
        result["cpu_baseline"], tests = cpu_baseline(frames, args.cpu_seconds)
        if args.cpu_seconds_one_core > 0:
            result["cpu_baseline_one_core"] = cpu_one_core(frames, args.cpu_seconds_one_core)
    result["kernels_ms"] = {k: float(np.mean([np.mean(v) for v in kernel_ms_frame[k]]))
                            for k in fvv.FRAME_KERNELS}
    if not args.no_gather:
        carve_ms = [float(np.mean(kernel_ms_frame["fine_carve"][f])) for f in range(len(masks))]
        result["gather_roofline"] = gather_leg(ctx, torch, sils, fine_vox, carve_ms, tests)

    # Rooflines of the two big kernels, from their own execution times (events
    # taken at each kernel's start and end on its stream, eager runs):
    #   fine carve:  per fine voxel 1 B of occupancy written, plus one 4-byte
    #                silhouette word per (voxel, camera) test of the index-order
    #                early exit (counted by the oracle on the same frames);
    #   exit points: per crossing edge 16 B written (key, xyz), plus one 4-byte
    #                word per (point, camera) test of the index-order early exit.
    # Both are gathers of 4-byte words from the cache-resident silhouettes, so
    # the bound is the measured gather rate BW_g (the fine carve's fraction of it
    # is its fraction of R_g = BW_g / (1 + 4 t)); hbm_frac is the same bytes
    # over the HBM peak.  The kernel with the longer time is "roofline".
    if tests:
        bw_g = result.get("gather_roofline", {}).get("bw_g_GBs")
        rl = {}
        for k, spec in KERNELS.items():
            ms = float(np.mean([np.mean(kernel_ms_frame[k][f]) for f in tests]))
            if k == "fine_carve":
                per = np.mean([tests[f]["vox"] + 4 * tests[f]["tests_fine"] for f in tests])
            else:
                per = np.mean([16 * tests[f]["edges"] + 4 * tests[f]["tests_surface"] for f in tests])
            achieved = per / (ms * 1e-3) / 1e9
            if bw_g:
                entry = {"kernel": spec["kernel"], "bound": "gather", "achieved": achieved,
                         "peak": bw_g, "unit": "GB/s", "frac": achieved / bw_g}
            else:
                entry = {"kernel": spec["kernel"], "bound": "hbm", "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS}
            entry.update({"traffic": stored_traffic(k), "bytes_per_launch": float(per),
                          "kernel_ms": ms, "hbm_frac": achieved / HBM_PEAK_GBS})
            rl[k] = entry
        dominant = max(rl, key=lambda k: rl[k]["kernel_ms"])
        result["roofline"] = rl[dominant]
        result["rooflines"] = rl
    print(json.dumps(result))


if __name__ == "__main__":
    main()
