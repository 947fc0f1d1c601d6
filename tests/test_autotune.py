"""Host logic of the batched-carve tile autotuner: the pixels-per-sample
figure of its cache key against a closed form, the key's fields and the JSON
cache round trip.  No GPU."""
import math

import numpy as np

from paper_1903_11785_amd import JOB_DTYPE, autotune


def pinhole(f, cx, cy):
    """Camera at the origin looking along +z (R = I, t = 0): P = K [I | 0]."""
    return np.array([[f, 0, cx, 0], [0, f, cy, 0], [0, 0, 1, 0]], np.float64)


def one_job(centre, h, dims=(9, 9, 9), n_cams=1, cam_base=0, W=320, H=240):
    j = np.zeros(1, JOB_DTYPE)
    d = np.asarray(dims)
    j[0]["h"] = h
    j[0]["origin"] = np.asarray(centre, np.float64) - (d - 1) / 2 * h
    j[0]["lo"] = (0, 0, 0)
    j[0]["dims"] = dims
    j[0]["n_cams"], j[0]["cam_base"] = n_cams, cam_base
    j[0]["width"], j[0]["height"] = W, H
    return j


def test_pixels_per_sample_closed_form():
    # on the optical axis at depth d, one lattice step h spans f*h/d pixels
    for f, d, h in [(300.0, 6.0, 0.01), (2000.0, 12.0, 0.01), (300.0, 3.0, 0.05)]:
        P = pinhole(f, 160.0, 120.0)[None]
        ppv = autotune.pixels_per_sample(P, one_job((0.0, 0.0, d), h))
        assert math.isclose(ppv, f * h / d, rel_tol=1e-6), (ppv, f * h / d)


def test_pixels_per_sample_off_axis_and_behind():
    # at x = z = d the projection is u = cx + f, and the figure is
    # h |row0 - u row2| / w = h |(f, 0, cx - u)| / d = f sqrt(2) h / d
    f, d, h = 300.0, 5.0, 0.01
    P = pinhole(f, 160.0, 120.0)[None]
    ppv = autotune.pixels_per_sample(P, one_job((d, 0.0, d), h))
    assert math.isclose(ppv, f * math.sqrt(2) * h / d, rel_tol=1e-6)
    # a camera that sees the job from behind contributes nothing
    assert autotune.pixels_per_sample(P, one_job((0.0, 0.0, -d), h)) == 0.0


def test_cache_key_fields_and_round_trip(tmp_path):
    P = np.stack([pinhole(300.0, 160.0, 120.0)] * 4)
    jobs = np.concatenate([one_job((0, 0, 6.0), 0.01, n_cams=4), one_job((0, 0, 6.0), 0.01, n_cams=4)])
    k = autotune.cache_key("gfx950", P, jobs)
    assert k.startswith("gfx950|n4|320x240|ppv")
    # 2 x 9^3 samples -> 2^11 bucket
    assert k.endswith("|v2^11")
    path = str(tmp_path / "c.json")
    autotune._store(path, {k: {"tx": 64, "tz": 4, "blocks": 2048, "ms": 1.5}})
    assert autotune._load(path)[k]["blocks"] == 2048
    assert autotune._load(str(tmp_path / "missing.json")) == {}


def test_default_candidates_are_valid_tiles():
    c = autotune.candidates(256)
    assert len(c) == len(autotune.CULLED_SHAPES) * len(autotune.GRID_MULTIPLES) + \
        len(autotune.PLAIN_SHAPES)
    for t in c:
        assert t.tx * t.ty == 256 and t.tx in (16, 32, 64) and t.tz in (1, 2, 4, 8)
        assert 0 < t.persistent_blocks <= (1 << 20)
