"""Tile autotuner of the batched fine carve (Sec. II-B-3 over many ROIs).

The bytes ``fvv_carve_batched`` writes do not depend on the tile; only its
speed does.  The best tile depends on:
- the camera count and image size;
- how many pixels one fine sample spans, which sets how often a 4x4x4 box of
  samples is decided by its corner rectangle alone;
- the amount of work.

The tuner times candidate tiles on the caller's own job table through
``fvv_tune_carve_batched`` (HIP events inside the library, one untimed call
per candidate first).  It keeps the winner in a JSON cache keyed by device
architecture, camera count, image size, a pixels-per-sample bucket and a
work bucket.  A cached key is not timed again.
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import JOB_DTYPE, Tile, tile

# (tx, tz) shapes and persistent-grid multiples of the CU count tried by default:
# depth 4 is the culled kernel (static XCD split), the others test every
# camera with dynamic tile grabbing.
CULLED_SHAPES = ((64, 4), (32, 4), (16, 4))
PLAIN_SHAPES = ((64, 1), (64, 2), (32, 2), (64, 8))
GRID_MULTIPLES = (8, 32, 64, 128)


def candidates(n_cus: int) -> List[Tile]:
    """Default candidate tiles for a device with n_cus compute units."""
    out = [tile(tx, tz, n_cus * m) for (tx, tz) in CULLED_SHAPES for m in GRID_MULTIPLES]
    out += [tile(tx, tz, n_cus * 8) for (tx, tz) in PLAIN_SHAPES]
    return out


def pixels_per_sample(P_table: np.ndarray, jobs: np.ndarray) -> float:
    """Median over (job, camera) of the image-space length of one lattice step
    at the job's box centre: h * |row0 - u row2| / w with u = row0.X / w."""
    P_table = np.asarray(P_table, np.float64).reshape(-1, 3, 4)
    jobs = np.asarray(jobs).view(JOB_DTYPE).reshape(-1)
    vals = []
    for j in jobs:
        h = float(j["h"])
        centre = (np.asarray(j["origin"], np.float64) +
                  (np.asarray(j["lo"], np.float64) + (np.asarray(j["dims"], np.float64) - 1) / 2) * h)
        Xh = np.append(centre, 1.0)
        for c in range(int(j["cam_base"]), int(j["cam_base"]) + int(j["n_cams"])):
            P = P_table[c]
            w = P[2] @ Xh
            if not w > 0:
                continue
            u = (P[0] @ Xh) / w
            vals.append(h * float(np.linalg.norm(P[0, :3] - u * P[2, :3])) / w)
    return float(np.median(vals)) if vals else 0.0


def cache_key(arch: str, P_table: np.ndarray, jobs: np.ndarray) -> str:
    jobs = np.asarray(jobs).view(JOB_DTYPE).reshape(-1)
    n = int(jobs["n_cams"].max())
    W, H = int(jobs["width"].max()), int(jobs["height"].max())
    ppv = pixels_per_sample(P_table, jobs)
    ppv_b = round(2 * math.log2(ppv)) / 2 if ppv > 0 else -99
    vox = float(np.prod(jobs["dims"].astype(np.float64), axis=1).sum())
    return f"{arch}|n{n}|{W}x{H}|ppv{ppv_b:+.1f}|v2^{round(math.log2(max(vox, 1.0)))}"


def _load(path: Optional[str]) -> Dict[str, dict]:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def _store(path: Optional[str], cache: Dict[str, dict]) -> None:
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_batched(ctx, jobs_host: np.ndarray, jobs_dev, cams_dev, P_table: np.ndarray, sils, out,
                 cache_path: Optional[str] = None, cands: Optional[Sequence[Tile]] = None,
                 reps: int = 3) -> dict:
    """Pick the tile of ``ctx.carve_batched`` for this job table.

    jobs_host: the job table as a JOB_DTYPE array (same as jobs_dev);
    P_table: the host copy of the camera table's P matrices [n][3][4];
    out: the output buffer (written by every timed call).
    Returns {"tile": Tile, "key", "cached", "table": [(tx, tz, blocks, ms), ...]}.
    cache_path defaults to $FVV_TUNE_CACHE (no cache when unset)."""
    import torch
    if cache_path is None:
        cache_path = os.environ.get("FVV_TUNE_CACHE") or None
    arch = torch.cuda.get_device_properties(sils.device).gcnArchName.split(":")[0]
    key = cache_key(arch, P_table, jobs_host)
    cache = _load(cache_path)
    if key in cache and cands is None:
        e = cache[key]
        return {"tile": tile(e["tx"], e["tz"], e["blocks"]), "key": key, "cached": True,
                "table": [(e["tx"], e["tz"], e["blocks"], e["ms"])]}
    n_cus = torch.cuda.get_device_properties(sils.device).multi_processor_count
    cands = list(cands) if cands is not None else candidates(n_cus)
    n_jobs = int(np.asarray(jobs_host).view(JOB_DTYPE).size)
    best, ms = ctx.tune_carve_batched(jobs_dev, n_jobs, cams_dev, sils, out, cands, reps=reps)
    table = [(c.tx, c.tz, c.persistent_blocks, m) for c, m in zip(cands, ms)]
    b = cands[best]
    cache[key] = {"tx": b.tx, "tz": b.tz, "blocks": b.persistent_blocks, "ms": ms[best]}
    _store(cache_path, cache)
    return {"tile": tile(b.tx, b.tz, b.persistent_blocks), "key": key, "cached": False,
            "table": table}
