"""Phase split of the labelling (Sec. II-B-2) on volleyball frames.

A measurement build of the library (``FVV_LABEL_PHASES`` defined) records the
GPU's real-time clock (100 MHz) at the end of each phase of the labelling
kernel.  ``--build`` compiles it to ``libfvv_label_phases.so`` beside the
library (no GPU needed); ``--run`` runs whole frames with it and prints, per
phase, the median time over the frames' repeated runs.

    python -m paper_1903_11785_amd.label_phases --build
    python -m paper_1903_11785_amd.label_phases --run --frames 4 --reps 20
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
PHASES_LIB = os.path.join(HERE, "libfvv_label_phases.so")
PHASES = ["row mask", "rows listed", "runs cut", "unions", "flatten + root numbers",
          "stats + Eq. (1) filter + ROIs", "labels + bitmap clear", "fine jobs laid out",
          "fine job radii"]
TICK_US = 0.01   # the real-time clock runs at 100 MHz


def build_phases() -> str:
    from . import build
    return build.build(defines=("FVV_LABEL_PHASES",), out=PHASES_LIB)


def run(frames: int, reps: int) -> dict:
    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import scenes
    import paper_1903_11785_amd as fvv
    if not os.path.exists(PHASES_LIB):
        raise SystemExit(f"{PHASES_LIB} is not built: run with --build first")
    fvv.LIB_PATH = PHASES_LIB          # the measurement build in place of the library
    L = fvv.library()
    L.fvv_label_phase_stamps.argtypes = [C.c_void_p, C.c_int32]
    L.fvv_label_phase_stamps.restype = C.c_int32
    torch.cuda.set_device(0)
    scs = [scenes.make_scene(scenes.CFG_VOLLEYBALL, f) for f in range(frames)]
    sc0 = scs[0]
    N, H, W = sc0.masks.shape
    coarse = fvv.Grid(origin=tuple(sc0.origin), h=sc0.hc, lo=(0, 0, 0), dims=sc0.coarse_dims)
    ctx = fvv.Context(max_cams=N, max_w=W, max_h=H, max_coarse=coarse.size, max_fine=1 << 26,
                      max_rois=256, max_points=1 << 22, max_jobs=256)
    params = fvv.frame_params(sc0.P32, W, H, coarse, sc0.hc_um, sc0.hf_um, sc0.t_np, sc0.t_nb,
                              sc0.n_steps)
    sils = torch.empty((N, H, (W + 31) // 32), dtype=torch.int32, device="cuda")
    bufs = fvv.FrameBuffers(coarse, 256, 1 << 26, 1 << 22)
    stamps = np.zeros(10, np.uint64)
    per = []
    for sc in scs:
        m = torch.from_numpy(sc.masks).cuda()
        for rep in range(reps + 1):
            ctx.frame(params, sils, bufs, masks=m)
            torch.cuda.synchronize()
            if L.fvv_label_phase_stamps(stamps.ctypes.data, 10) != 0:
                raise RuntimeError("no phase stamps")
            if rep:
                per.append(np.diff(stamps.astype(np.int64)) * TICK_US)
    if ctx.check() != fvv.FVV_OK:
        raise RuntimeError("frame exceeded a capacity")
    per = np.array(per)
    med = np.median(per, axis=0)
    out = {"workload": f"volleyball, {frames} frames x {reps} runs", "unit": "us",
           "phases": {p: round(float(v), 2) for p, v in zip(PHASES, med)},
           "total_us": round(float(np.median(per.sum(axis=1))), 2)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--build", action="store_true")
    ap.add_argument("--run", action="store_true")
    ap.add_argument("--frames", type=int, default=4)
    ap.add_argument("--reps", type=int, default=20)
    a = ap.parse_args()
    if a.build:
        print(build_phases())
    if a.run:
        print(json.dumps(run(a.frames, a.reps), indent=1))


if __name__ == "__main__":
    main()
