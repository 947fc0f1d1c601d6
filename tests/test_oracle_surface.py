"""Pins of the oracle's ROI lattices and surface step.

ROI (Sec. II-B-3, each ROI becomes its own fine volume): the integer mapping
against Python's exact integer arithmetic, and containment of the dilated box.
Edges (Sec. II-C, edges whose endpoints differ): brute force with numpy.
Exit points (Sec. II-C, Eq. (2)-(3), first exit over all cameras):
  P-S1  bisection t* against the exact FP64 first exit, found by walking the
        pixel-boundary crossings of the edge in every camera (perspective-
        correct, so no image-space ratio), on edges with a single transition;
  P-S2  the point lies within 0.5 px of a foreground pixel in every camera and
        of a background pixel in at least one;
  P-S3  the point lies outside the solid eroded by the pixel footprint.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import scenes

GUARD_PX = 1e-3


# ------------------------------------------------------------------ ROI lattices
def py_roi(coarse_lo, coarse_n, hc, hf, blo, bhi):
    lo, n = [], []
    for a in range(3):
        A = coarse_lo[a] + blo[a] - 1
        B = coarse_lo[a] + bhi[a] + 1
        f0 = (A * hc) // hf
        f1 = -((-(B * hc)) // hf)
        fmin = -((-(coarse_lo[a] * hc)) // hf)
        fmax = ((coarse_lo[a] + coarse_n[a] - 1) * hc) // hf
        f0, f1 = max(f0, fmin), min(f1, fmax)
        lo.append(f0)
        n.append(f1 - f0 + 1)
    return tuple(lo), tuple(n)


def test_roi_integer_mapping_against_python():
    rng = np.random.default_rng(3)
    for _ in range(3000):
        hc = int(rng.choice([62500, 100000, 40000, 50000, 80000, 33333]))
        hf = int(rng.choice([20000, 10000, 5000, 15000, 7000, 1000]))
        clo = tuple(int(v) for v in rng.integers(-40, 40, 3))
        cn = tuple(int(v) for v in rng.integers(1, 200, 3))
        blo = [int(rng.integers(0, c)) for c in cn]
        bhi = [int(rng.integers(b, c)) for b, c in zip(blo, cn)]
        coarse = oracle.Lattice(origin=np.zeros(3, np.float32), h=np.float32(hc * 1e-6), lo=clo, dims=cn)
        got = oracle.roi_fine(coarse, hc, hf, np.float32(hf * 1e-6), blo, bhi)
        assert (got.lo, got.dims) == py_roi(clo, cn, hc, hf, blo, bhi)


def test_roi_contains_dilated_box():
    """Every fine sample whose exact position lies in the one-cell dilation of
    the coarse box (and inside the coarse lattice's extent) is in the ROI."""
    hc, hf = 62500, 20000
    coarse = oracle.Lattice(origin=np.zeros(3, np.float32), h=np.float32(0.0625), lo=(0, 0, 0),
                            dims=(64, 64, 32))
    blo, bhi = (8, 35, 10), (17, 48, 20)
    got = oracle.roi_fine(coarse, hc, hf, np.float32(0.02), blo, bhi)
    for a in range(3):
        lo_um = max((blo[a] - 1) * hc, 0)
        hi_um = min((bhi[a] + 1) * hc, (coarse.dims[a] - 1) * hc)
        need = [g for g in range(-5, 400) if lo_um <= g * hf <= hi_um]
        assert got.lo[a] <= need[0] and need[-1] <= got.lo[a] + got.dims[a] - 1
        assert got.lo[a] * hf >= lo_um - hf and (got.lo[a] + got.dims[a] - 1) * hf <= hi_um + hf


# ------------------------------------------------------------------ edges
def brute_edges(occ):
    o = occ != 0
    nz, ny, nx = o.shape
    keys = []
    for axis, (sl0, sl1) in enumerate([((slice(None), slice(None), slice(0, -1)),
                                        (slice(None), slice(None), slice(1, None))),
                                       ((slice(None), slice(0, -1), slice(None)),
                                        (slice(None), slice(1, None), slice(None))),
                                       ((slice(0, -1), slice(None), slice(None)),
                                        (slice(1, None), slice(None), slice(None)))]):
        d = o[sl0] != o[sl1]
        k, j, i = np.nonzero(d)
        keys.append(3 * (i + nx * (j + ny * k)).astype(np.int64) + axis)
    return np.sort(np.concatenate(keys))


@pytest.mark.parametrize("seed", range(6))
def test_edges_brute_force(seed):
    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in rng.integers(1, 20, 3))
    occ = (rng.uniform(size=shape) < [0.1, 0.5, 0.9][seed % 3]).astype(np.uint8)
    np.testing.assert_array_equal(oracle.edges(occ).astype(np.int64), brute_edges(occ))


def test_edges_degenerate():
    assert oracle.edges(np.zeros((4, 5, 6), np.uint8)).size == 0
    assert oracle.edges(np.ones((4, 5, 6), np.uint8)).size == 0
    one = np.zeros((1, 1, 2), np.uint8)
    one[0, 0, 1] = 1
    assert oracle.edges(one).tolist() == [0]


# ------------------------------------------------------------------ exit points
def _pixel_fg(mask, x, y):
    H, W = mask.shape
    if not (0 <= x < W and 0 <= y < H):
        return False
    return bool(mask[int(np.floor(y)), int(np.floor(x))])


def exact_first_exit(sc, lat, occ, key):
    """FP64 first exit along the edge, or None if the combined predicate does not
    have exactly one inside->outside transition (or disagrees at the ends)."""
    nx, ny, nz = lat.dims
    lin, axis = divmod(int(key), 3)
    g = np.array([lat.lo[0] + lin % nx, lat.lo[1] + (lin // nx) % ny, lat.lo[2] + lin // (nx * ny)],
                 np.float64)
    stride = [1, nx, nx * ny][axis]
    p_on = occ.reshape(-1)[lin] != 0
    g_on = g.copy()
    if not p_on:
        g_on[axis] += 1
    d = 1.0 if p_on else -1.0
    h, o = float(lat.h), np.asarray(lat.origin, np.float64)
    X0 = g_on * h + o
    X1 = X0.copy()
    X1[axis] += d * h
    cuts = {0.0, 1.0}
    proj = []
    for c in range(sc.P32.shape[0]):
        P = sc.P32[c].astype(np.float64)
        a0, b0, w0 = P @ np.append(X0, 1.0)
        a1, b1, w1 = P @ np.append(X1, 1.0)
        if w0 <= 0 or w1 <= 0:
            return None
        proj.append((a0, b0, w0, a1, b1, w1))
        for (u0, u1) in ((a0, a1), (b0, b1)):
            lo_v, hi_v = sorted((u0 / w0, u1 / w1))
            for nint in range(int(np.floor(lo_v)) + 1, int(np.floor(hi_v)) + 1):
                den = (u1 - u0) - nint * (w1 - w0)
                if den != 0:
                    t = (nint * w0 - u0) / den
                    if 0 < t < 1:
                        cuts.add(t)
    cuts = sorted(cuts)

    def inside(t):
        res = True
        for c, (a0, b0, w0, a1, b1, w1) in enumerate(proj):
            a, b, w = a0 + t * (a1 - a0), b0 + t * (b1 - b0), w0 + t * (w1 - w0)
            x, y = a / w, b / w
            if min(abs(x - round(x)), abs(y - round(y))) < GUARD_PX:
                return None              # the edge runs along a pixel edge: fp32 may pick either side
            res = res and _pixel_fg(sc.masks[c], x, y)
        return res

    states = [inside(0.5 * (t0 + t1)) for t0, t1 in zip(cuts[:-1], cuts[1:])]
    if any(s is None for s in states):
        return None
    if not states[0] or states[-1]:
        return None
    first_out = states.index(False)
    if any(states[first_out:]):
        return None
    return cuts[first_out]


def _surface(sc):
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims)
    assert len(res.keys) >= 1
    return res


@pytest.mark.parametrize("frame", [0, 3])
def test_ps1_bisection_matches_exact_first_exit(scene_cache, frame):
    sc = scene_cache(1, frame)
    res = _surface(sc)
    rng = np.random.default_rng(frame)
    checked = strict = 0
    for lat, occ, keys, t_star in zip(res.fine, res.occ_fine, res.keys, res.tstar):
        pick = rng.choice(keys.size, size=min(400, keys.size), replace=False)
        for e in pick:
            t_ex = exact_first_exit(sc, lat, occ, keys[e])
            if t_ex is None:
                continue
            checked += 1
            # fp32 projection error is ~1e-4 px, under 2e-4 of an edge of the tiny rig's
            # fine lattice (>= 0.6 px): only an exit that close to a bisection midpoint
            # k/256 may be bracketed on the other side of it
            near_dyadic = abs(t_ex * 256 - round(t_ex * 256)) < 256 * 2e-4
            tol = 2.0 ** -9 + (2e-4 if near_dyadic else 1e-7)
            strict += not near_dyadic
            assert abs(float(t_star[e]) - t_ex) <= tol, (e, float(t_star[e]), t_ex)
    assert checked > 300 and strict > 0.8 * checked


def _near_pixels(mask, x, y, r=0.5):
    """Values of the pixels whose squares lie within distance r of (x, y);
    off-image squares count as background."""
    H, W = mask.shape
    vals = []
    for yi in range(int(np.floor(y - r)), int(np.floor(y + r)) + 1):
        for xi in range(int(np.floor(x - r)), int(np.floor(x + r)) + 1):
            dx = max(xi - x, 0.0, x - (xi + 1))
            dy = max(yi - y, 0.0, y - (yi + 1))
            if dx * dx + dy * dy <= r * r:
                vals.append(bool(mask[yi, xi]) if (0 <= xi < W and 0 <= yi < H) else False)
    return vals


@pytest.mark.parametrize("cfg,frame", [(1, 1), (2, 0)])
def test_ps2_points_within_half_pixel_of_boundary(scene_cache, cfg, frame):
    sc = scene_cache(cfg, frame)
    res = _surface(sc)
    rng = np.random.default_rng(7)
    for xyz in res.xyz:
        pick = xyz[rng.choice(xyz.shape[0], size=min(300, xyz.shape[0]), replace=False)].astype(np.float64)
        for X in pick:
            some_bg = False
            for c, cam in enumerate(sc.cams):
                P = sc.P32[c].astype(np.float64)
                a, b, w = P @ np.append(X, 1.0)
                vals = _near_pixels(sc.masks[c], a / w, b / w)
                assert any(vals), "no foreground pixel within 0.5 px"
                some_bg |= not all(vals)
            assert some_bg, "no background pixel within 0.5 px in any camera"


@pytest.mark.parametrize("cfg,frame", [(1, 2), (2, 0)])
def test_ps3_points_outside_eroded_solid(scene_cache, cfg, frame):
    sc = scene_cache(cfg, frame)
    res = _surface(sc)
    for lat, xyz in zip(res.fine, res.xyz):
        X = xyz.astype(np.float64)
        depth = np.stack([scenes.project64(c, X)[2] for c in sc.cams])
        f = np.array([c.K[0, 0] for c in sc.cams])[:, None]
        r = (0.71 * depth / f).max(axis=0) + 1e-4 + float(lat.h) / 256
        for e in sc.ellipsoids:
            s = np.clip(1.0 - r / e.axes.min(), 0.0, None)
            d = X - e.center
            assert not np.any(np.einsum('ni,ij,nj->n', d, e.M, d) <= s * s)


@pytest.mark.parametrize("cfg,frame", [(1, 0), (1, 3)])
def test_bisection_brackets_are_consistent(scene_cache, cfg, frame):
    """Sec. II-C, Eq. (3): bisection keeps the exit inside its bracket.  The
    reported parameter is a dyadic midpoint (2k+1)/2^(S+1), so the final
    bracket is [t* - 2^-(S+1), t* + 2^-(S+1)]; its lower end is 0 or a point
    the occupancy test finds inside, its upper end 1 or a point it finds
    outside (points formed exactly as the bisection forms them)."""
    sc = scene_cache(cfg, frame)
    res = _surface(sc)
    S = sc.n_steps
    half = np.float32(2.0 ** -(S + 1))
    checked = 0
    for lat, occ, keys, t in zip(res.fine, res.occ_fine, res.keys, res.tstar):
        k = t.astype(np.float64) * 2.0 ** (S + 1)
        assert np.all(k == np.round(k)) and np.all(np.round(k) % 2 == 1)
        for e in range(0, keys.size, max(1, keys.size // 300)):
            lo, hi = t[e] - half, t[e] + half
            if lo > 0:
                X = oracle.edge_point(lat, occ, int(keys[e]), lo)
                assert oracle.point_inside(sc.P32, res.sils, sc.W, sc.H, *X), (e, lo)
            if hi < 1:
                X = oracle.edge_point(lat, occ, int(keys[e]), hi)
                assert not oracle.point_inside(sc.P32, res.sils, sc.W, sc.H, *X), (e, hi)
            checked += 1
    assert checked > 100


def test_edge_point_ends_are_the_lattice_samples(scene_cache):
    """The edge point at t = 0 is the occupied endpoint and at t = 1 the other
    one, each coordinate the lattice value fma((float)g, h, o) rounded once."""
    sc = scene_cache(1, 0)
    res = _surface(sc)
    lat, occ, keys = res.fine[0], res.occ_fine[0], res.keys[0]
    nx, ny, _ = lat.dims
    flat = occ.reshape(-1)
    for e in range(0, keys.size, max(1, keys.size // 100)):
        lin, axis = divmod(int(keys[e]), 3)
        g = np.array([lin % nx, (lin // nx) % ny, lin // (nx * ny)])
        g2 = g.copy()
        g2[axis] += 1
        on, off = (g, g2) if flat[lin] else (g2, g)
        for t, s in ((0.0, on), (1.0, off)):
            want = [_fma32(lat.lo[a] + int(s[a]), lat.h, lat.origin[a]) for a in range(3)]
            assert np.array_equal(oracle.edge_point(lat, occ, int(keys[e]), t),
                                  np.array(want, np.float32))


def _fma32(g, h, o) -> np.float32:
    """float32 fma((float)g, h, o): the exact value g*h + o correctly rounded
    (to nearest, ties to even) to float32."""
    v = Fraction(float(np.float32(g))) * Fraction(float(np.float32(h))) + \
        Fraction(float(np.float32(o)))
    x = np.float32(float(v))
    cands = [np.nextafter(x, np.float32(-np.inf)), x, np.nextafter(x, np.float32(np.inf))]
    return min(cands, key=lambda c: (abs(Fraction(float(c)) - v),
                                     int(np.array(c, np.float32).view(np.uint32)) & 1))


def test_bisection_test_count_bounds(scene_cache):
    """The bisection's (point, camera) test count of the index-order early exit:
    every step tests at least the first camera and at most all of them, and
    with a single camera exactly one per step."""
    sc = scene_cache(1, 0)
    res = _surface(sc)
    lat, occ, keys = res.fine[0], res.occ_fine[0], res.keys[0]
    E, S, N = keys.size, sc.n_steps, sc.P32.shape[0]
    _, _, T = oracle.bisect(sc.P32, res.sils, sc.W, sc.H, lat, occ, keys, S, count_tests=True)
    assert E > 0 and S * E <= T <= S * E * N
    _, _, T1 = oracle.bisect(sc.P32[:1], res.sils[:1], sc.W, sc.H, lat, occ, keys, S,
                             count_tests=True)
    assert T1 == S * E
