"""Time splits of the labelling (Sec. II-B-2) and of the fine carve
(Sec. II-B-3) on volleyball frames, from a measurement build.

The measurement build of the library (``FVV_LABEL_PHASES`` and
``FVV_CARVE_PROBE`` defined) records the GPU's real-time clock (100 MHz):

* at the end of each phase of the labelling kernel (its one workgroup);
* for every wave of the fine carve, its entry and exit, and for each of its
  first blocks of 16 x 4 x 4 samples the block's start and end, its test
  passes and its (sub-block, camera) tests.

``--build`` compiles it to ``libfvv_measure.so`` beside the library (no GPU
needed); ``--run`` runs whole frames with it and prints both splits as JSON.

    python -m paper_1903_11785_amd.phase_split --build
    python -m paper_1903_11785_amd.phase_split --run --frames 4 --reps 20
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
MEASURE_LIB = os.path.join(HERE, "libfvv_measure.so")
DEFINES = ("FVV_LABEL_PHASES", "FVV_CARVE_PROBE")
LABEL_PHASES = ["row mask", "rows listed", "runs cut", "pairs listed", "unions",
                "flatten + root numbers",
                "stats + Eq. (1) filter + ROIs", "labels", "fine jobs laid out",
                "fine job radii"]
N_STAMPS = len(LABEL_PHASES) + 1
PROBE_WAVES, PROBE_ITERS = 16384, 4       # the probe tables of the measurement build
TICK_US = 0.01                            # the real-time clock runs at 100 MHz


def build_measure() -> str:
    from . import build
    return build.build(defines=DEFINES, out=MEASURE_LIB)


def carve_split(blocks: np.ndarray, waves: np.ndarray) -> dict:
    """The fine carve's time split from one run's probe tables."""
    wv = waves[waves[:, 0] != 0]
    base = int(wv[:, 0].min())
    ent = (wv[:, 0].astype(np.int64) - base) * TICK_US
    ext = (wv[:, 1].astype(np.int64) - base) * TICK_US
    n_blk = (wv[:, 2] & 0xffffffff).astype(np.int64)
    tables = (wv[:, 2] >> 32).astype(np.int64) * TICK_US
    b = blocks.reshape(PROBE_WAVES, PROBE_ITERS, 3)
    used = b[:, :, 0] != 0
    st = (b[:, :, 0].astype(np.int64) - base) * TICK_US
    en = (b[:, :, 1].astype(np.int64) - base) * TICK_US
    dur = np.where(used, en - st, 0.0)
    passes = (b[:, :, 2] & 0xffff).astype(np.int64)
    tests = (b[:, :, 2] >> 16).astype(np.int64)
    widx = np.nonzero(waves[:, 0] != 0)[0]
    # a wave's time before its first block, between its blocks, after its last
    first = st[widx, 0] - ent
    has = used[widx, 0]
    gaps = []
    for k in range(1, PROBE_ITERS):
        m = used[widx, k]
        gaps.append((st[widx, k] - en[widx, k - 1])[m])
    gaps = np.concatenate(gaps) if gaps else np.zeros(0)
    d = dur[used]
    p = passes[used]
    classes = {}
    for lo, hi, name in ((0, 1, "no test pass"), (1, 4, "1-3 passes"), (4, 8, "4-7 passes"),
                         (8, 1 << 16, "8+ passes")):
        m = (p >= lo) & (p < hi)
        classes[name] = {"blocks": int(m.sum()), "mean_us": round(float(d[m].mean()), 2) if m.any() else 0.0,
                         "share_of_block_time": round(float(d[m].sum() / d.sum()), 3)}
    span = float(ext.max())
    wave_time = float((ext - ent).sum())
    return {
        "span_us": round(span, 2),
        "waves": int(len(wv)),
        "blocks_recorded": int(used.sum()),
        "blocks_total": int(n_blk.sum()),
        "block_us": {"mean": round(float(d.mean()), 2), "p50": round(float(np.median(d)), 2),
                     "p99": round(float(np.percentile(d, 99)), 2), "max": round(float(d.max()), 2)},
        "blocks_by_passes": classes,
        "tests_per_block_mean": round(float(tests[used].mean()), 2),
        "wave_time_split": {
            "before_first_block": round(float(first[has].sum() / wave_time), 3),
            "in_blocks": round(float(d.sum() / wave_time), 3),
            "between_blocks": round(float(gaps.sum() / wave_time), 3),
        },
        "before_first_block_us_mean": round(float(first[has].mean()), 2),
        "of_which_tables_and_barrier_us_mean": round(float(tables[has].mean()), 2),
        "between_blocks_us_mean": round(float(gaps.mean()), 2) if gaps.size else 0.0,
        "wave_entry_us": {"p50": round(float(np.median(ent)), 2), "max": round(float(ent.max()), 2)},
        "busy_fraction_of_span": round(wave_time / (span * 256 * 28), 3),
    }


def run(frames: int, reps: int, cfg: str = "volleyball") -> dict:
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import scenes
    import paper_1903_11785_amd as fvv
    if not os.path.exists(MEASURE_LIB):
        raise SystemExit(f"{MEASURE_LIB} is not built: run with --build first")
    fvv.LIB_PATH = MEASURE_LIB          # the measurement build in place of the library
    L = fvv.library()
    L.fvv_label_phase_stamps.argtypes = [C.c_void_p, C.c_int32]
    L.fvv_label_phase_stamps.restype = C.c_int32
    L.fvv_carve_probe_read.argtypes = [C.c_void_p, C.c_void_p]
    L.fvv_carve_probe_read.restype = C.c_int32
    L.fvv_carve_probe_clear.argtypes = []
    L.fvv_carve_probe_clear.restype = C.c_int32
    torch.cuda.set_device(0)
    cfg_id = {"volleyball": scenes.CFG_VOLLEYBALL, "judo": scenes.CFG_JUDO,
              "paper_volleyball": scenes.CFG_PAPER_V}[cfg]
    scs = [scenes.make_scene(cfg_id, f) for f in range(frames)]
    sc0 = scs[0]
    N, H, W = sc0.masks.shape
    coarse = fvv.Grid(origin=tuple(sc0.origin), h=sc0.hc, lo=(0, 0, 0), dims=sc0.coarse_dims)
    ctx = fvv.Context(max_cams=N, max_w=W, max_h=H, max_coarse=coarse.size, max_fine=1 << 27,
                      max_rois=256, max_points=1 << 23, max_jobs=256)
    params = fvv.frame_params(sc0.P32, W, H, coarse, sc0.hc_um, sc0.hf_um, sc0.t_np, sc0.t_nb,
                              sc0.n_steps)
    sils = torch.empty((N, H, (W + 31) // 32), dtype=torch.int32, device="cuda")
    bufs = fvv.FrameBuffers(coarse, 256, 1 << 27, 1 << 23)
    stamps = np.zeros(N_STAMPS, np.uint64)
    blocks = np.zeros((PROBE_WAVES * PROBE_ITERS, 3), np.uint64)
    waves = np.zeros((PROBE_WAVES, 3), np.uint64)
    label, carve = [], []
    for sc in scs:
        m = torch.from_numpy(sc.masks).cuda()
        for rep in range(reps + 1):
            if L.fvv_carve_probe_clear() != 0:
                raise RuntimeError("probe tables not cleared")
            ctx.frame(params, sils, bufs, masks=m)
            torch.cuda.synchronize()
            if L.fvv_label_phase_stamps(stamps.ctypes.data, N_STAMPS) != 0:
                raise RuntimeError("no phase stamps")
            if L.fvv_carve_probe_read(blocks.ctypes.data, waves.ctypes.data) != 0:
                raise RuntimeError("no carve probe")
            if rep:
                label.append(np.diff(stamps.astype(np.int64)) * TICK_US)
                carve.append(carve_split(blocks, waves))
    if ctx.check() != fvv.FVV_OK:
        raise RuntimeError("frame exceeded a capacity")
    label = np.array(label)
    med = np.median(label, axis=0)
    # the fine carve: the run with the median span
    carve.sort(key=lambda c: c["span_us"])
    return {
        "workload": f"{cfg}, {frames} frames x {reps} runs",
        "labelling_us": {p: round(float(v), 2) for p, v in zip(LABEL_PHASES, med)},
        "labelling_total_us": round(float(np.median(label.sum(axis=1))), 2),
        "fine_carve_median_run": carve[len(carve) // 2],
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--build", action="store_true")
    ap.add_argument("--run", action="store_true")
    ap.add_argument("--frames", type=int, default=4)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--cfg", default="volleyball", choices=["volleyball", "judo", "paper_volleyball"])
    a = ap.parse_args()
    if a.build:
        print(build_measure())
    if a.run:
        print(json.dumps(run(a.frames, a.reps, a.cfg), indent=1))


if __name__ == "__main__":
    main()
