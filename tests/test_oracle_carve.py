"""Pins of the oracle's occupancy test (paper Sec. II-B: a voxel is unoccupied
when its projection falls outside a silhouette; occupied iff inside all).

P-C1  analytic FP64 agreement: recompute every voxel's pixel in FP64 and look
      it up in the unpacked analytic masks; disagreements only inside a 1e-3 px
      guard band around pixel edges.
P-C2  containment: the hull contains the solid eroded by the pixel footprint.
P-C3  tightening: more cameras never add voxels (nested camera sets).
P-C4  special cases: empty / full silhouettes, a camera looking away.
"""
import numpy as np
import pytest

import oracle
import scenes

GUARD_PX = 1e-3


def lattice_points(lat):
    nx, ny, nz = lat.dims
    g = np.stack(np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij"), -1)
    g = g[..., ::-1].astype(np.float64) + np.asarray(lat.lo, np.float64)      # (i, j, k) + lo
    return g * float(lat.h) + np.asarray(lat.origin, np.float64)            # [nz][ny][nx][3]


def fp64_occupancy(P32, masks, X):
    """AND over cameras of the analytic silhouette at the FP64 pixel of X, and a
    flag marking voxels within GUARD_PX of a pixel edge in some camera."""
    N, H, W = masks.shape
    occ = np.ones(X.shape[:-1], bool)
    near = np.zeros(X.shape[:-1], bool)
    Xh = np.concatenate([X, np.ones(X.shape[:-1] + (1,))], -1)
    for c in range(N):
        P = P32[c].astype(np.float64)
        a, b, w = (Xh @ P.T).transpose(-1, *range(X.ndim - 1))
        ok = w > 0
        x = np.where(ok, a / np.where(ok, w, 1), -1)
        y = np.where(ok, b / np.where(ok, w, 1), -1)
        near |= (np.abs(x - np.round(x)) < GUARD_PX) | (np.abs(y - np.round(y)) < GUARD_PX)
        inside = ok & (x >= 0) & (x < W) & (y >= 0) & (y < H)
        xi = np.clip(np.floor(x), 0, W - 1).astype(np.int64)
        yi = np.clip(np.floor(y), 0, H - 1).astype(np.int64)
        occ &= inside & (masks[c][yi, xi] != 0)
    return occ, near


def _coarse(sc):
    return oracle.Lattice(origin=sc.origin, h=sc.hc, lo=(0, 0, 0), dims=sc.coarse_dims)


@pytest.mark.parametrize("cfg,frame", [(1, 0), (1, 1), (1, 2), (1, 3), (2, 0)])
def test_pc1_analytic_agreement_coarse(scene_cache, cfg, frame):
    sc = scene_cache(cfg, frame)
    lat = _coarse(sc)
    occ, _ = oracle.carve(sc.P32, oracle.pack(sc.masks), sc.W, sc.H, lat)
    ref, near = fp64_occupancy(sc.P32, sc.masks, lattice_points(lat))
    diff = (occ != 0) != ref
    assert ref.sum() > 0
    assert not np.any(diff & ~near), f"{int((diff & ~near).sum())} disagreements outside the guard band"


@pytest.mark.parametrize("frame", [0, 1, 2])
def test_pc1_analytic_agreement_fine_roi(scene_cache, frame):
    sc = scene_cache(1, frame)
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims, surface=False)
    assert len(res.fine) >= 1
    for lat, occ in zip(res.fine, res.occ_fine):
        ref, near = fp64_occupancy(sc.P32, sc.masks, lattice_points(lat))
        diff = (occ != 0) != ref
        assert not np.any(diff & ~near)


def _eroded_inside(sc, X):
    """Points whose distance to every ellipsoid's surface exceeds the pixel
    footprint r = max_c 0.71 z_c / f_c + 1e-4 m (scaled-ellipsoid erosion).  X is
    a lattice ([nz][ny][nx][3], ascending coordinates): each ellipsoid is
    evaluated on the lattice points of its bounding cube only."""
    out = np.zeros(X.shape[:-1], bool)
    axes = (X[0, 0, :, 0], X[0, :, 0, 1], X[:, 0, 0, 2])
    f = np.array([c.K[0, 0] for c in sc.cams]).reshape(-1, 1, 1, 1)
    for e in sc.ellipsoids:
        a = float(e.axes.max())
        (i0, i1), (j0, j1), (k0, k1) = (
            (int(np.searchsorted(v, e.center[t] - a)),
             int(np.searchsorted(v, e.center[t] + a, side="right")))
            for t, v in enumerate(axes))
        if i0 >= i1 or j0 >= j1 or k0 >= k1:
            continue
        Xs = X[k0:k1, j0:j1, i0:i1]
        depth = np.stack([scenes.project64(c, Xs)[2] for c in sc.cams])
        r = (0.71 * depth / f).max(axis=0) + 1e-4
        s = np.clip(1.0 - r / e.axes.min(), 0.0, None)
        d = Xs - e.center
        out[k0:k1, j0:j1, i0:i1] |= np.einsum('...i,ij,...j->...', d, e.M, d) <= s * s
    return out


@pytest.mark.parametrize("cfg,frame", [(1, 0), (1, 5), (2, 0)])
def test_pc2_hull_contains_eroded_solid(scene_cache, cfg, frame):
    sc = scene_cache(cfg, frame)
    lat = _coarse(sc)
    occ, _ = oracle.carve(sc.P32, oracle.pack(sc.masks), sc.W, sc.H, lat)
    inside = _eroded_inside(sc, lattice_points(lat))
    assert inside.sum() > 10
    assert np.all(occ[inside] == 1)


def test_pc3_tightening_with_nested_camera_sets():
    sphere = [scenes.Ellipsoid(center=np.zeros(3), Q=np.eye(3), axes=np.full(3, 0.5))]
    lat = oracle.Lattice(origin=np.float32([-1, -1, -1]), h=np.float32(0.03125), lo=(0, 0, 0),
                         dims=(64, 64, 64))
    X = lattice_points(lat)
    prev, counts = None, []
    true_inside = np.einsum('...i,...i->...', X, X) <= 0.25
    for n in (1, 2, 4, 8, 16, 32):
        rig = scenes.tiny_rig(n)
        masks = scenes.render_masks(rig, sphere)
        P = np.stack([c.P32 for c in rig])
        occ, _ = oracle.carve(P, oracle.pack(masks), 320, 240, lat)
        occ = occ.astype(bool)
        counts.append(int(occ.sum()))
        if prev is not None:
            assert not np.any(occ & ~prev), f"{n} cameras added voxels"
        prev = occ
    assert all(a >= b for a, b in zip(counts, counts[1:]))
    assert counts[-1] >= int(true_inside.sum()) * 0.9
    assert counts[0] > counts[-1]


def test_pc4_empty_and_full_silhouettes(scene_cache):
    sc = scene_cache(1, 0)
    lat = _coarse(sc)
    zero = np.zeros_like(sc.masks)
    occ, T = oracle.carve(sc.P32, oracle.pack(zero), sc.W, sc.H, lat)
    assert occ.sum() == 0 and T == lat.size            # every voxel rejected by camera 0
    full = np.ones_like(sc.masks)
    wide = oracle.Lattice(origin=np.float32([-7, -7, -4]), h=np.float32(0.25), lo=(0, 0, 0),
                          dims=(56, 56, 32))            # reaches behind the cameras and off-image
    occ, _ = oracle.carve(sc.P32, oracle.pack(full), sc.W, sc.H, wide)
    ref, near = fp64_occupancy(sc.P32, full, lattice_points(wide))
    assert not np.any(((occ != 0) != ref) & ~near)
    assert 0 < occ.sum() < wide.size


def test_pc4_camera_looking_away_carves_everything(scene_cache):
    sc = scene_cache(1, 0)
    lat = _coarse(sc)
    away = scenes.look_at([8.0, 0.0, 0.0], [16.0, 0.0, 0.0], 300.0, 320, 240)   # volume behind it
    P = np.concatenate([sc.P32, away.P32[None]], 0)
    masks = np.concatenate([sc.masks, np.ones((1, 240, 320), np.uint8)], 0)
    occ, _ = oracle.carve(P, oracle.pack(masks), 320, 240, lat)
    assert occ.sum() == 0


def test_tests_count_is_index_order_early_exit(scene_cache):
    """T = sum over voxels of (index of the first rejecting camera + 1, or N)."""
    sc = scene_cache(1, 2)
    lat = oracle.Lattice(origin=sc.origin, h=sc.hc, lo=(10, 12, 4), dims=(20, 17, 9))
    sils = oracle.pack(sc.masks)
    occ, T = oracle.carve(sc.P32, sils, sc.W, sc.H, lat)
    X = lattice_points(lat)
    N = sc.P32.shape[0]
    alive = np.ones(X.shape[:-1], bool)
    T_ref = 0
    for c in range(N):
        T_ref += int(alive.sum())
        occ_c, _ = fp64_occupancy(sc.P32[c:c + 1], sc.masks[c:c + 1], X)
        alive &= occ_c
    assert T == T_ref
    np.testing.assert_array_equal(occ.astype(bool), alive)
