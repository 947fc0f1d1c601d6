"""Pins of the oracle's Bresenham isovalue (oracle.isovalue, Sec. II-C,
Eq. (2)-(3) as the paper computes them).

  - single-camera ratios of Eq. (2) on hand-built silhouettes: horizontal,
    reversed, vertical and diagonal lines against a straight boundary, a line
    that leaves the image, an all-foreground line, a background start pixel,
    a first step onto background;
  - the traced pixels are those of the ideal line: with one background pixel
    placed on the ideal line (the pixel nearest to it at some step along the
    major axis, away from rounding ties), the ratio is the one of the nearest
    pixel one step earlier;
  - whole edges on a ball seen by three cameras with ~6-8 px edges, against
    the exact FP64 first exit of Eq. (3)'s minimum (perspective-correct, from
    pixel-boundary crossings): the estimate is quantised to pixels and traced
    between floored end pixels, so it is within 1.5 px (over the edge's pixel
    length) for nearly all edges -- lines grazing the silhouette boundary can
    be off by more -- close on average, and early on average (the last
    foreground pixel precedes the exit); a reversed walk (mean error ~0.5) or
    a ratio taken at the first background pixel (late on average) fails;
  - lambda in [0, 1) on every crossing edge and its point on the edge.
"""
import types

import numpy as np
import pytest

import oracle
import scenes
from test_oracle_surface import exact_first_exit


def sil_from(fg, W, H):
    """Packed single silhouette from a predicate fg(x, y) on pixel indices."""
    y, x = np.mgrid[:H, :W]
    mask = fg(x, y).astype(np.uint8)[None]
    return oracle.pack(mask)[0]


@pytest.mark.parametrize("fg,W,H,p_on,p_off,expect", [
    (lambda x, y: x <= 7, 32, 10, (2, 5), (12, 5), 25 / 100),          # P_i = (7, 5)
    (lambda x, y: x >= 8, 32, 10, (14, 5), (2, 5), 36 / 144),          # walking left, P_i = (8, 5)
    (lambda x, y: y <= 3, 10, 12, (4, 0), (4, 9), 9 / 81),             # P_i = (4, 3)
    (lambda x, y: x + y <= 6, 10, 10, (0, 0), (6, 6), 18 / 72),        # P_i = (3, 3)
    (lambda x, y: x >= 0, 40, 40, (3, 4), (30, 21), 1.0),              # all foreground
    (lambda x, y: x >= 0, 8, 6, (5, 2), (10, 2), 4 / 25),              # leaves the image at x = 8
    (lambda x, y: x > 100, 16, 16, (3, 3), (9, 9), 0.0),               # start pixel background
    (lambda x, y: x <= 3, 16, 16, (3, 3), (4, 3), 0.0),                # first step is background
    (lambda x, y: x >= 0, 16, 16, (3, 3), (3, 3), 1.0),                # one pixel
])
def test_line_ratio_hand_cases(fg, W, H, p_on, p_off, expect):
    sil = sil_from(fg, W, H)
    assert oracle.line_lambda2(sil, W, H, p_on, p_off) == pytest.approx(expect, rel=0, abs=1e-15)


def test_traced_pixels_follow_the_ideal_line():
    rng = np.random.default_rng(3)
    W = H = 96
    checked = 0
    for _ in range(400):
        p0 = rng.integers(10, 86, 2)
        p1 = rng.integers(10, 86, 2)
        d = p1 - p0
        major = int(np.argmax(np.abs(d)))
        L = int(abs(d[major]))
        if L < 3:
            continue
        minor = 1 - major
        m = int(rng.integers(2, L + 1))        # step of the background pixel

        def nearest(k):
            t = k / L
            v = p0[minor] + t * d[minor]
            if abs((v % 1.0) - 0.5) < 0.1:       # near a rounding tie: either pixel is right
                return None
            px = np.empty(2, np.int64)
            px[major] = p0[major] + np.sign(d[major]) * k
            px[minor] = int(np.floor(v + 0.5))
            return px

        bg, before = nearest(m), nearest(m - 1)
        if bg is None or before is None:
            continue
        sil = sil_from(lambda x, y: ~((x == bg[0]) & (y == bg[1])), W, H)
        got = oracle.line_lambda2(sil, W, H, p0, p1)
        want = float(np.sum((before - p0) ** 2)) / float(np.sum(d ** 2))
        assert got == pytest.approx(want, rel=0, abs=1e-15), (p0, p1, m)
        checked += 1
    assert checked > 200


def ball_scene():
    """A 0.25 m ball at the origin, three 400x400 cameras at 2 m, f = 1000 px,
    and a 20 mm lattice over it (edges of ~6-8 px in every camera)."""
    dirs = [(1.0, 1.0, 0.5), (-1.0, 1.0, 0.7), (0.3, -1.0, 0.9)]
    cams = []
    for d in dirs:
        d = np.asarray(d) / np.linalg.norm(d)
        cams.append(scenes.look_at(2.0 * d, np.zeros(3), 1000.0, 400, 400))
    ball = scenes.Ellipsoid(center=np.zeros(3), Q=np.eye(3), axes=np.full(3, 0.25))
    masks = scenes.render_masks(cams, [ball])
    P32 = np.stack([c.P32 for c in cams])
    lat = oracle.Lattice(origin=np.full(3, -0.4, np.float32), h=np.float32(0.02), lo=(0, 0, 0),
                         dims=(41, 41, 41))
    return types.SimpleNamespace(P32=P32, masks=masks, W=400, H=400, cams=cams), lat


def test_lambda_tracks_the_exact_first_exit():
    sc, lat = ball_scene()
    sils = oracle.pack(sc.masks)
    occ, _ = oracle.carve(sc.P32, sils, sc.W, sc.H, lat)
    keys = oracle.edges(occ)
    lam, xyz = oracle.isovalue(sc.P32, sils, sc.W, sc.H, lat, occ, keys)
    assert keys.size > 2000
    errs = []
    nx, ny, _ = lat.dims
    for e in range(0, keys.size, 3):
        t_ex = exact_first_exit(sc, lat, occ, keys[e])
        if t_ex is None:
            continue
        # shortest pixel length of the edge over the cameras
        lin, axis = divmod(int(keys[e]), 3)
        g = np.array([lin % nx, (lin // nx) % ny, lin // (nx * ny)], np.float64)
        X0 = lat.origin.astype(np.float64) + g * float(lat.h)
        X1 = X0.copy()
        X1[axis] += float(lat.h)
        L = min(np.hypot(*(c.P64 @ np.append(X1, 1))[:2] / (c.P64 @ np.append(X1, 1))[2]
                         - (c.P64 @ np.append(X0, 1))[:2] / (c.P64 @ np.append(X0, 1))[2])
                for c in sc.cams)
        assert L > 5.0
        errs.append((float(lam[e]) - t_ex, L))
    errs = np.array(errs)
    assert len(errs) > 500
    d, L = errs[:, 0], errs[:, 1]
    assert np.mean(np.abs(d) * L <= 1.5) > 0.97
    assert np.mean(np.abs(d)) < 0.1
    assert -0.12 < np.mean(d) < 0.0


def test_lambda_range_and_points_on_the_edges(scene_cache):
    sc = scene_cache(1, 0)
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims)
    sils = oracle.pack(sc.masks)
    for lat, occ, keys in zip(res.fine, res.occ_fine, res.keys):
        lam, xyz = oracle.isovalue(sc.P32, sils, sc.W, sc.H, lat, occ, keys)
        assert (lam >= 0).all() and (lam < 1).all()
        nx, ny, _ = lat.dims
        lin, axis = keys // 3, keys % 3
        g = np.stack([lat.lo[0] + lin % nx, lat.lo[1] + (lin // nx) % ny,
                      lat.lo[2] + lin // (nx * ny)], 1).astype(np.float64)
        X0 = g * float(lat.h) + lat.origin.astype(np.float64)
        rows = np.arange(keys.size)
        lo_ax = X0[rows, axis]
        hi_ax = lo_ax + float(lat.h)
        pt = xyz[rows, axis].astype(np.float64)
        assert ((pt >= lo_ax - 1e-6) & (pt <= hi_ax + 1e-6)).all()
        # the other two coordinates are the lattice values
        for a in range(3):
            off = axis != a
            np.testing.assert_allclose(xyz[off, a], X0[off, a], rtol=0, atol=1e-6)
