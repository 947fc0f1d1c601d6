"""GPU parity: the HIP path through the C ABI against the CPU oracle, element by
element on the same seeded inputs.  Occupancy, labels, ROI boxes and edge keys
must be bit-exact (0 mismatches); exit points must agree within 1e-4 of the
fine voxel edge (both sides compute the same dyadic parameter, so they are
expected to agree exactly).  Sizes span several tiles with ragged tails, up to
the full volleyball and judo frames."""
import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.gpu

TILES = [(tx, tz) for tx in (64, 32, 16) for tz in (1, 2, 4, 8)]


@pytest.fixture(scope="module")
def fvv():
    import paper_1903_11785_amd as fvv
    return fvv


@pytest.fixture(scope="module")
def ctx(fvv):
    c = fvv.Context(max_coarse=5_000_000, max_fine=1 << 28, max_rois=4096, max_points=1 << 23,
                    max_jobs=4096)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def sils_dev(ctx, masks):
    s = ctx.pack_silhouettes(dev(masks))
    return s


def grid_of(fvv, lat):
    return fvv.Grid(origin=tuple(np.float32(lat.origin)), h=np.float32(lat.h), lo=tuple(lat.lo),
                    dims=tuple(lat.dims))


def coarse_lat(sc):
    return oracle.Lattice(origin=sc.origin, h=sc.hc, lo=(0, 0, 0), dims=sc.coarse_dims)


# ------------------------------------------------------------------ packing
@pytest.mark.parametrize("shape", [(4, 240, 320), (3, 7, 33), (2, 5, 31), (1, 3, 64), (5, 9, 100)])
def test_pack(ctx, shape):
    rng = np.random.default_rng(sum(shape))
    masks = (rng.uniform(size=shape) < 0.5).astype(np.uint8) * rng.integers(1, 255, size=shape).astype(np.uint8)
    got = host(ctx.pack_silhouettes(dev(masks))).view(np.uint32)
    np.testing.assert_array_equal(got, oracle.pack(masks))


def test_pack_full_frames(ctx, scene_cache):
    for cfg in (2, 3):
        sc = scene_cache(cfg, 0)
        got = host(ctx.pack_silhouettes(dev(sc.masks))).view(np.uint32)
        np.testing.assert_array_equal(got, oracle.pack(sc.masks))


# ------------------------------------------------------------------ carving
@pytest.mark.parametrize("tx,tz", TILES)
def test_carve_tiny_coarse_every_tile(fvv, ctx, scene_cache, tx, tz):
    sc = scene_cache(1, 0)
    lat = coarse_lat(sc)
    ref, _ = oracle.carve(sc.P32, oracle.pack(sc.masks), sc.W, sc.H, lat)
    got = host(ctx.carve(sc.P32, sc.W, sc.H, sils_dev(ctx, sc.masks), grid_of(fvv, lat),
                         fvv.tile(tx, tz)))
    assert int((got != ref).sum()) == 0


@pytest.mark.parametrize("seed", range(1, 7))
def test_carve_tiny_coarse_and_fine(fvv, ctx, scene_cache, seed):
    sc = scene_cache(1, seed)
    sils = sils_dev(ctx, sc.masks)
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims, surface=False)
    got = host(ctx.carve(sc.P32, sc.W, sc.H, sils, grid_of(fvv, res.coarse)))
    assert int((got != res.occ_coarse).sum()) == 0
    for lat, ref in zip(res.fine, res.occ_fine):
        got = host(ctx.carve(sc.P32, sc.W, sc.H, sils, grid_of(fvv, lat), fvv.tile(32, 2)))
        assert int((got != ref).sum()) == 0


@pytest.mark.parametrize("cfg", [2, 3])
def test_carve_full_size_coarse(fvv, ctx, scene_cache, cfg):
    sc = scene_cache(cfg, 0)
    lat = coarse_lat(sc)
    ref, _ = oracle.carve(sc.P32, oracle.pack(sc.masks), sc.W, sc.H, lat)
    got = host(ctx.carve(sc.P32, sc.W, sc.H, sils_dev(ctx, sc.masks), grid_of(fvv, lat),
                         fvv.tile(64, 1)))
    assert int((got != ref).sum()) == 0


def test_carve_integer_quotients(fvv, ctx):
    """Projections that land exactly on pixel edges (a/w integral), where a
    rounded quotient floors to the wrong pixel unless corrected exactly."""
    rng = np.random.default_rng(5)
    W = H = 160
    for scale in (3.0, 0.1, 7.0, 1.0 / 3.0, 13.0):
        s = np.float32(scale)
        P = np.array([[[s, 0, 0, 0], [0, s, 0, 0], [0, 0, 0, s]],
                      [[0, s, 0, s], [0, 0, s, 0], [0, 0, 0, s]]], np.float32)
        masks = (rng.uniform(size=(2, H, W)) < 0.7).astype(np.uint8)
        lat = oracle.Lattice(origin=np.float32([-1, -1, 0]), h=np.float32(0.25), lo=(0, 0, 0),
                             dims=(300, 7, 300))
        ref, _ = oracle.carve(P, oracle.pack(masks), W, H, lat)
        got = host(ctx.carve(P, W, H, sils_dev(ctx, masks), grid_of(fvv, lat), fvv.tile(64, 4)))
        assert int((got != ref).sum()) == 0
        assert 0 < ref.sum() < ref.size


def test_carve_behind_and_off_image(fvv, ctx, scene_cache):
    sc = scene_cache(1, 0)
    away = scenes.look_at([3.0, 0.0, 0.0], [16.0, 0.0, 0.0], 300.0, 320, 240)
    P = np.concatenate([sc.P32, away.P32[None]], 0)
    masks = np.concatenate([sc.masks, np.ones((1, 240, 320), np.uint8)], 0)
    lat = oracle.Lattice(origin=np.float32([-7, -7, -4]), h=np.float32(0.125), lo=(0, 0, 0),
                         dims=(112, 112, 64))
    for cams in (slice(0, 4), slice(0, 5), slice(4, 5)):
        ref, _ = oracle.carve(P[cams], oracle.pack(masks[cams]), 320, 240, lat)
        got = host(ctx.carve(P[cams], 320, 240, sils_dev(ctx, masks[cams]), grid_of(fvv, lat)))
        assert int((got != ref).sum()) == 0


def test_carve_negative_lattice_indices_and_ragged(fvv, ctx, scene_cache):
    sc = scene_cache(1, 3)
    sils = sils_dev(ctx, sc.masks)
    for lo, dims in [((-37, -20, -9), (131, 61, 47)), ((3, -50, 1), (65, 129, 3)),
                     ((0, 0, 0), (1, 1, 1)), ((-100, -100, -50), (1, 257, 9))]:
        lat = oracle.Lattice(origin=np.float32([0.3, -0.2, 0.1]), h=np.float32(0.02), lo=lo,
                             dims=dims)
        ref, _ = oracle.carve(sc.P32, oracle.pack(sc.masks), sc.W, sc.H, lat)
        for tx, tz in ((64, 4), (16, 8), (32, 1)):
            got = host(ctx.carve(sc.P32, sc.W, sc.H, sils, grid_of(fvv, lat), fvv.tile(tx, tz)))
            assert int((got != ref).sum()) == 0


# ------------------------------------------------------------------ labelling
def check_label(fvv, ctx, occ, t_np=1, t_nb=0xFFFFFFFF, max_rois=4096):
    nz, ny, nx = occ.shape
    g = fvv.Grid(origin=(0, 0, 0), h=1.0, lo=(0, 0, 0), dims=(nx, ny, nz))
    occ_d = dev(occ.astype(np.uint8))
    labels, rois, n = ctx.label(g, occ_d, t_np, t_nb, max_rois)
    ref_occ, ref_lab, ref_rois, K = oracle.label(occ, t_np, t_nb)
    assert int(host(n)[0]) == K
    np.testing.assert_array_equal(host(labels), ref_lab)
    np.testing.assert_array_equal(host(occ_d), ref_occ)
    k = min(K, max_rois)
    np.testing.assert_array_equal(host(rois)[:k], ref_rois[:k])
    return K


@pytest.mark.parametrize("seed", range(10))
def test_label_random(fvv, ctx, seed):
    rng = np.random.default_rng(100 + seed)
    shape = tuple(int(v) for v in rng.integers(5, 70, size=3))
    dens = [0.03, 0.1, 0.2, 0.35, 0.5][seed % 5]
    occ = (rng.uniform(size=shape) < dens).astype(np.uint8)
    check_label(fvv, ctx, occ)
    check_label(fvv, ctx, occ, t_np=3, t_nb=50)


def test_label_adversarial_shapes(fvv, ctx):
    occ = np.zeros((37, 41, 45), np.uint8)
    for t in range(37):
        occ[t, t, t] = 1                      # diagonal through many blocks, vertex contacts only
    occ[0, 40, 0:45:2] = 1                    # isolated voxels along a row
    k, j, i = np.indices((20, 20, 40))
    cb = ((i + j + k) % 2 == 0).astype(np.uint8)
    spiral = np.zeros((8, 64, 64), np.uint8)
    y, x = 32, 32
    for s in range(1, 60):
        for _ in range(s):
            x += 1 if s % 2 else -1
            if 0 <= x < 64:
                spiral[s % 8, y, x] = 1
        for _ in range(s):
            y += 1 if s % 2 else -1
            if 0 <= y < 64 and 0 <= x < 64:
                spiral[s % 8, y, x] = 1
    for g in (occ, cb, spiral, np.ones((9, 10, 33), np.uint8), np.zeros((3, 4, 5), np.uint8)):
        check_label(fvv, ctx, g)


def test_label_repeated_merge_orders(fvv, ctx):
    """Shapes whose unions race: a comb (teeth joining one spine in parallel), a
    rake (separate columns joined only by their last row), 3-D staircases with
    vertex contacts, and dense random fields in LDS and past it (global forest);
    each labelled 12 times, every run byte-identical to the oracle."""
    comb = np.zeros((24, 8, 120), np.uint8)
    comb[0, 4, :] = 1
    comb[:, 4, 0::2] = 1
    rake = np.zeros((30, 6, 96), np.uint8)
    rake[:, 2, 0::3] = 1
    rake[29, 2, :] = 1
    stairs = np.zeros((40, 40, 40), np.uint8)
    for t in range(40):
        stairs[t, t, (t * 7) % 40] = 1
        stairs[t, 39 - t, t] = 1
    rng = np.random.default_rng(7)
    dense = (rng.uniform(size=(12, 32, 48)) < 0.5).astype(np.uint8)   # ~4.6e3 runs: LDS
    big = (rng.uniform(size=(48, 64, 96)) < 0.45).astype(np.uint8)    # ~7.4e4 runs: global
    for g in (comb, rake, stairs, dense, big):
        for _ in range(12):
            check_label(fvv, ctx, g)


def test_label_filter_bounds(fvv, ctx):
    occ = np.zeros((10, 10, 30), np.uint8)
    occ[1, 1, 0:3] = 1
    occ[5, 5, 0:4] = 1
    occ[8, 8, 10:15] = 1
    occ[1, 8, 20:26] = 1
    for t_np, t_nb in [(4, 5), (3, 6), (5, 5), (7, 0xFFFFFFFF), (1, 3)]:
        check_label(fvv, ctx, occ, t_np, t_nb)


def test_label_capacity_overflow(fvv, ctx):
    occ = np.zeros((6, 6, 12), np.uint8)
    occ[0, 0, 0] = occ[3, 3, 3] = occ[5, 5, 8] = 1
    assert ctx.check() == fvv.FVV_OK
    K = check_label(fvv, ctx, occ, max_rois=2)
    assert K == 3
    assert ctx.check() == fvv.FVV_ECAPACITY
    assert ctx.check() == fvv.FVV_OK


@pytest.mark.parametrize("cfg,frame", [(1, 0), (1, 4), (2, 0), (3, 0)])
def test_label_scene_coarse(fvv, ctx, scene_cache, cfg, frame):
    sc = scene_cache(cfg, frame)
    occ, _ = oracle.carve(sc.P32, oracle.pack(sc.masks), sc.W, sc.H, coarse_lat(sc))
    check_label(fvv, ctx, occ, sc.t_np, sc.t_nb)


# ------------------------------------------------------------------ surface
def check_surface(fvv, ctx, sc, lat, occ, sils, steps=8, max_points=1 << 22):
    keys_ref = oracle.edges(occ)
    xyz_ref, _ = oracle.bisect(sc.P32, oracle.pack(sc.masks), sc.W, sc.H, lat, occ, keys_ref, steps)
    keys, xyz, n = ctx.surface(grid_of(fvv, lat), dev(occ), sc.P32, sc.W, sc.H, sils, steps,
                               max_points)
    E = int(host(n)[0])
    assert E == keys_ref.size
    k = min(E, max_points)
    np.testing.assert_array_equal(host(keys)[:k].view(np.uint32), keys_ref[:k])
    err = np.abs(host(xyz)[:k].astype(np.float64) - xyz_ref[:k].astype(np.float64)).max(initial=0)
    assert err <= 1e-4 * float(lat.h)
    return E, err


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_surface_tiny(fvv, ctx, scene_cache, seed):
    sc = scene_cache(1, seed)
    sils = sils_dev(ctx, sc.masks)
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims, surface=False)
    for lat, occ in zip(res.fine, res.occ_fine):
        for steps in (8, 1, 12):
            E, err = check_surface(fvv, ctx, sc, lat, occ, sils, steps)
            assert E > 0 and err == 0.0


def test_surface_degenerate_and_capacity(fvv, ctx, scene_cache):
    sc = scene_cache(1, 0)
    sils = sils_dev(ctx, sc.masks)
    lat = oracle.Lattice(origin=sc.origin, h=sc.hf, lo=(90, 90, 40), dims=(1, 1, 1))
    E, _ = check_surface(fvv, ctx, sc, lat, np.zeros((1, 1, 1), np.uint8), sils)
    assert E == 0
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims, surface=False)
    lat, occ = res.fine[0], res.occ_fine[0]
    assert ctx.check() == fvv.FVV_OK
    E, _ = check_surface(fvv, ctx, sc, lat, occ, sils, max_points=1000)
    assert E > 1000
    assert ctx.check() == fvv.FVV_ECAPACITY


# ------------------------------------------------------------------ batched carve
def batched_case(n_frames=3, rois_per_frame=4, scale=0.35):
    sc_list, boxes = scenes.batched_rois(n_frames, rois_per_frame, hf_um=20000,
                                         edge_lo=0.6 * scale * 2, edge_hi=2.5 * scale * 2)
    return sc_list, boxes


def batched_inputs(fvv, ctx, scs, boxes):
    W, H = scs[0].W, scs[0].H
    N = scs[0].P32.shape[0]
    P_all = np.concatenate([s.P32 for s in scs], 0)
    sils = sils_dev(ctx, np.concatenate([s.masks for s in scs], 0))
    cams_dev = fvv.cameras_to_device(P_all, W, H)
    jobs, total = fvv.frame_major_jobs([(b.frame, b.lo, b.dims) for b in boxes],
                                       [s.origin for s in scs], [s.hf for s in scs], N, W, H)
    return P_all, sils, cams_dev, jobs, fvv.jobs_to_device(jobs), total


# culled (depth 4, static XCD split; grids rounded up to whole XCD rounds) and
# plain (dynamic grabbing) tiles, with grids from one workgroup up
BATCHED_TILES = [(64, 4, 0), (32, 4, 5), (16, 4, 1), (32, 2, 7), (16, 8, 1), (64, 1, 3000)]


def test_batched_equals_per_roi_and_oracle(fvv, ctx):
    import torch
    scs, boxes = batched_case()
    P_all, sils, cams_dev, jobs, jobs_d, total = batched_inputs(fvv, ctx, scs, boxes)
    W, H = scs[0].W, scs[0].H
    outs = []
    for (tx, tz, blocks) in BATCHED_TILES:
        out = torch.full((total,), 7, dtype=torch.uint8, device="cuda")
        ctx.carve_batched(jobs_d, len(boxes), cams_dev, sils, out, fvv.tile(tx, tz, blocks))
        outs.append(host(out))
    assert ctx.check() == fvv.FVV_OK
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    for t, b in enumerate(boxes):
        s = scs[b.frame]
        lat = oracle.Lattice(origin=s.origin, h=s.hf, lo=b.lo, dims=b.dims)
        ref, _ = oracle.carve(s.P32, oracle.pack(s.masks), W, H, lat)
        seg = outs[0][int(jobs[t]["out_offset"]):int(jobs[t]["out_offset"]) + lat.size]
        assert int((seg.reshape(ref.shape) != ref).sum()) == 0
        per = host(ctx.carve(s.P32, W, H, sils_dev(ctx, s.masks), grid_of(fvv, lat)))
        np.testing.assert_array_equal(per, ref)


def test_batched_graph_replays(fvv, ctx):
    """The captured batched carve equals the eager call on every replay, with
    the output reset and other eager work in between."""
    import torch
    scs, boxes = batched_case(n_frames=2, rois_per_frame=3)
    P_all, sils, cams_dev, jobs, jobs_d, total = batched_inputs(fvv, ctx, scs, boxes)
    ref = torch.full((total,), 7, dtype=torch.uint8, device="cuda")
    ctx.carve_batched(jobs_d, len(boxes), cams_dev, sils, ref)
    for (tx, tz, blocks) in [(64, 4, 0), (32, 2, 0)]:
        out = torch.full((total,), 7, dtype=torch.uint8, device="cuda")
        g = ctx.carve_batched_graph(jobs_d, len(boxes), cams_dev, sils, out,
                                    fvv.tile(tx, tz, blocks))
        for rep in range(3):
            out.fill_(9)
            other = torch.full((total,), 5, dtype=torch.uint8, device="cuda")
            ctx.carve_batched(jobs_d, len(boxes), cams_dev, sils, other, fvv.tile(16, 1, 3))
            g.launch(torch.cuda.current_stream())
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (tx, tz, rep)
            assert torch.equal(other, ref)
        g.close()
    assert ctx.check() == fvv.FVV_OK


def test_batched_autotuner(fvv, ctx, tmp_path):
    """The tuner times every candidate, returns the fastest, caches it under
    its key, and leaves the (tile-independent) output in place."""
    import torch
    from paper_1903_11785_amd import autotune
    scs, boxes = batched_case(n_frames=2, rois_per_frame=3)
    P_all, sils, cams_dev, jobs, jobs_d, total = batched_inputs(fvv, ctx, scs, boxes)
    ref = torch.full((total,), 7, dtype=torch.uint8, device="cuda")
    ctx.carve_batched(jobs_d, len(boxes), cams_dev, sils, ref)
    out = torch.full((total,), 7, dtype=torch.uint8, device="cuda")
    cache = str(tmp_path / "tune.json")
    cands = [fvv.tile(64, 4, 256), fvv.tile(32, 2, 512), fvv.tile(16, 4, 64)]
    r = autotune.tune_batched(ctx, jobs, jobs_d, cams_dev, P_all, sils, out, cache_path=cache,
                              cands=cands, reps=2)
    assert not r["cached"] and len(r["table"]) == 3
    ms = [row[3] for row in r["table"]]
    assert all(m > 0 for m in ms)
    best = int(np.argmin(ms))
    assert (r["tile"].tx, r["tile"].tz) == (cands[best].tx, cands[best].tz)
    assert torch.equal(out, ref)
    r2 = autotune.tune_batched(ctx, jobs, jobs_d, cams_dev, P_all, sils, out, cache_path=cache)
    assert r2["cached"] and r2["key"] == r["key"]
    assert (r2["tile"].tx, r2["tile"].tz) == (r["tile"].tx, r["tile"].tz)
    assert ctx.check() == fvv.FVV_OK


def test_batched_skips_invalid_jobs(fvv, ctx):
    """A job out of range is not carved (its bytes stay untouched), the others
    are, and the next check reports EINVAL."""
    import torch
    scs, boxes = batched_case(n_frames=1, rois_per_frame=3)
    P_all, sils, cams_dev, jobs, jobs_d, total = batched_inputs(fvv, ctx, scs, boxes)
    ref = torch.full((total,), 7, dtype=torch.uint8, device="cuda")
    ctx.carve_batched(jobs_d, len(boxes), cams_dev, sils, ref)
    assert ctx.check() == fvv.FVV_OK
    bad = jobs.copy()
    bad[1]["n_cams"] = fvv.MAX_CAMS + 1
    bad_d = fvv.jobs_to_device(bad)
    a, b = int(jobs[1]["out_offset"]), int(jobs[2]["out_offset"])
    for (tx, tz) in [(64, 4), (32, 2)]:
        out = torch.full((total,), 7, dtype=torch.uint8, device="cuda")
        ctx.carve_batched(bad_d, len(boxes), cams_dev, sils, out, fvv.tile(tx, tz, 0))
        assert ctx.check() == fvv.FVV_EINVAL
        o, r = host(out), host(ref)
        assert (o[a:b] == 7).all()
        np.testing.assert_array_equal(o[:a], r[:a])
        np.testing.assert_array_equal(o[b:], r[b:])
    assert ctx.check() == fvv.FVV_OK


def test_batched_full_workload(fvv, ctx):
    """The batched workload at full size (64 frames x 12 uneven ROIs at 1 cm,
    2.9e9 samples) in the launch the benchmark times: the graph of the culled
    batched carve equals 768 per-ROI fvv_carve launches of the unculled carve
    (depth-2 tiles test every camera at every sample, so they share no
    classification code with the culled kernels) byte for byte, every ROI of
    the first four frames (48 ROIs, 1.7e8 samples) equals the oracle byte for
    byte, and sampled sub-boxes of every 16th ROI of the others equal it too."""
    import torch
    scs, boxes = scenes.batched_rois()
    P_all, sils, cams_dev, jobs, jobs_d, total = batched_inputs(fvv, ctx, scs, boxes)
    W, H = scs[0].W, scs[0].H
    print(f"batched full: {len(boxes)} ROIs, {total} samples", flush=True)
    out = torch.full((total,), 7, dtype=torch.uint8, device="cuda")
    g = ctx.carve_batched_graph(jobs_d, len(boxes), cams_dev, sils, out)
    g.launch(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g.close()
    assert ctx.check() == fvv.FVV_OK
    per = torch.full((total,), 7, dtype=torch.uint8, device="cuda")
    unculled = fvv.tile(64, 2)
    for t, b in enumerate(boxes):
        s = scs[b.frame]
        o = int(jobs[t]["out_offset"])
        n = int(np.prod(b.dims))
        grid = fvv.Grid(origin=tuple(np.float32(s.origin)), h=np.float32(s.hf), lo=tuple(b.lo),
                        dims=tuple(b.dims))
        ctx.carve(s.P32, W, H, sils[b.frame * 4:(b.frame + 1) * 4], grid, tile_=unculled,
                  out=per[o:o + n])
    torch.cuda.synchronize()
    assert ctx.check() == fvv.FVV_OK
    assert torch.equal(out, per)
    del per
    # every ROI of frames 0-3 against the oracle, whole
    packed = {}
    for t, b in enumerate(boxes):
        if b.frame >= 4:
            continue
        s = scs[b.frame]
        if b.frame not in packed:
            packed[b.frame] = oracle.pack(s.masks)
        lat = oracle.Lattice(origin=s.origin, h=s.hf, lo=tuple(b.lo), dims=tuple(b.dims))
        ref, _ = oracle.carve(s.P32, packed[b.frame], W, H, lat)
        o = int(jobs[t]["out_offset"])
        got = host(out[o:o + lat.size]).reshape(ref.shape)
        assert np.array_equal(got, ref), f"ROI {t} (frame {b.frame}) differs from the oracle"
    rng = np.random.default_rng(11)
    for t in range(0, len(boxes), 16):
        b = boxes[t]
        if b.frame < 4:
            continue
        s = scs[b.frame]
        nx, ny, nz = b.dims
        sub = (min(16, nx), min(16, ny), min(8, nz))
        i0, j0, k0 = (int(rng.integers(0, d - e + 1)) for d, e in zip(b.dims, sub))
        lat = oracle.Lattice(origin=s.origin, h=s.hf, lo=(b.lo[0] + i0, b.lo[1] + j0, b.lo[2] + k0),
                             dims=sub)
        ref, _ = oracle.carve(s.P32, oracle.pack(s.masks), W, H, lat)
        o = int(jobs[t]["out_offset"])
        seg = out[o:o + nx * ny * nz].view(nz, ny, nx)[k0:k0 + sub[2], j0:j0 + sub[1],
                                                        i0:i0 + sub[0]]
        np.testing.assert_array_equal(host(seg), ref)


# ------------------------------------------------------------------ whole frame
def run_frame(fvv, ctx, sc, max_rois=256, max_fine=1 << 26, max_points=1 << 22, graph=False,
              pack_first=False, coarse_tile=None, fine_tile=None, sils_fill=0):
    coarse = fvv.Grid(origin=tuple(sc.origin), h=sc.hc, lo=(0, 0, 0), dims=sc.coarse_dims)
    params = fvv.frame_params(sc.P32, sc.W, sc.H, coarse, sc.hc_um, sc.hf_um, sc.t_np, sc.t_nb,
                              sc.n_steps, coarse_tile=coarse_tile, fine_tile=fine_tile)
    bufs = fvv.FrameBuffers(coarse, max_rois, max_fine, max_points)
    import torch
    masks = dev(sc.masks)
    N, H, W = sc.masks.shape
    sils = torch.full((N, H, (W + 31) // 32), sils_fill, dtype=torch.int32, device="cuda")
    if graph:                                  # packing inside the graph
        g = ctx.frame_graph(params, sils, bufs, masks=masks)
        return g, bufs, sils
    if pack_first:                             # packed by a separate call
        ctx.pack_silhouettes(masks, out=sils)
        ctx.frame(params, sils, bufs)
    else:
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(fvv.FRAME_EVENTS)]
        ctx.frame(params, sils, bufs, masks=masks, events=ev)
        torch.cuda.synchronize()
        assert all(ev[i].elapsed_time(ev[i + 1]) >= 0
                   for i in range(fvv.FRAME_STAGE_EVENTS - 1))
        # each kernel's own time lies inside its stage's
        for q, stage in enumerate(fvv.FRAME_KERNELS):
            s = fvv.STAGES.index(stage)
            k0, k1 = ev[fvv.FRAME_STAGE_EVENTS + 2 * q], ev[fvv.FRAME_STAGE_EVENTS + 2 * q + 1]
            assert 0 < k0.elapsed_time(k1) <= ev[s].elapsed_time(ev[s + 1])
    return None, bufs, sils


def compare_frame(fvv, sc, bufs, res):
    counts = host(bufs.counts)
    K = len(res.rois)
    assert int(counts[0]) == K and int(counts[3]) == K
    np.testing.assert_array_equal(host(bufs.occ_coarse), res.occ_filtered)
    np.testing.assert_array_equal(host(bufs.labels), res.labels)
    np.testing.assert_array_equal(host(bufs.rois)[:K], res.rois)
    jobs = bufs.jobs_host(K)
    occ_fine = host(bufs.occ_fine)
    keys = host(bufs.keys).view(np.uint32)
    xyz = host(bufs.xyz)
    poff = host(bufs.point_off)
    assert int(counts[1]) == res.fine_voxels
    assert int(counts[2]) == sum(k.size for k in res.keys)
    for t, lat in enumerate(res.fine):
        assert tuple(jobs[t]["lo"]) == lat.lo and tuple(jobs[t]["dims"]) == lat.dims
        assert np.float32(jobs[t]["h"]) == lat.h
        o = int(jobs[t]["out_offset"])
        seg = occ_fine[o:o + lat.size].reshape(res.occ_fine[t].shape)
        assert int((seg != res.occ_fine[t]).sum()) == 0
        a, b = int(poff[t]), int(poff[t + 1])
        np.testing.assert_array_equal(keys[a:b], res.keys[t])
        err = np.abs(xyz[a:b].astype(np.float64) - res.xyz[t].astype(np.float64)).max(initial=0)
        assert err <= 1e-4 * float(lat.h)


@pytest.mark.parametrize("cfg,frame", [(1, 0), (1, 1), (1, 2), (2, 0), (2, 1), (3, 0), (3, 1)])
def test_frame_against_oracle(fvv, ctx, scene_cache, cfg, frame):
    sc = scene_cache(cfg, frame)
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims, sc.t_np,
                       sc.t_nb, sc.n_steps)
    _, bufs, sils = run_frame(fvv, ctx, sc, pack_first=(frame % 2 == 1))
    assert ctx.check() == fvv.FVV_OK
    compare_frame(fvv, sc, bufs, res)
    np.testing.assert_array_equal(host(sils).view(np.uint32), oracle.pack(sc.masks))


@pytest.mark.parametrize("width", [312, 316, 320])
def test_frame_ragged_width(fvv, ctx, scene_cache, width):
    """Images cut at the right edge: a width of 8k pixels that is not a row of
    whole 32-bit words (the one-pass packing of rows and 8 x 8 blocks clears
    the row's padding bytes), one that is not a multiple of 8 (rows and blocks
    packed in turn) and the full width."""
    import dataclasses
    sc = scene_cache(1, 0)
    masks = np.ascontiguousarray(sc.masks[:, :, :width])
    # foreground noise along the cut edge, so that the last bits of every row
    # matter; the silhouette buffer starts all ones, so that every bit the
    # packing leaves unwritten shows
    rng = np.random.default_rng(width)
    masks[:, :, -12:] = (rng.uniform(size=masks[:, :, -12:].shape) < 0.5).astype(np.uint8) * 255
    sc = dataclasses.replace(sc, masks=masks,
                             cams=[dataclasses.replace(c, W=width) for c in sc.cams])
    assert sc.W == width and sc.masks.shape[2] == width
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims, sc.t_np,
                       sc.t_nb, sc.n_steps)
    _, bufs, sils = run_frame(fvv, ctx, sc, sils_fill=-1)
    assert ctx.check() == fvv.FVV_OK
    compare_frame(fvv, sc, bufs, res)
    np.testing.assert_array_equal(host(sils).view(np.uint32), oracle.pack(sc.masks))


def many_balls_scene():
    """72 separate balls (r = 0.1 m, 6 x 6 x 2 on a 0.55 m grid) seen by 8 cameras of
    the tiny ring: 72 ROIs, more than one wave's worth for the fine-job layout."""
    rig = scenes.tiny_rig(8)
    ells = [scenes.Ellipsoid(center=np.array([(i - 2.5) * 0.55, (j - 2.5) * 0.55, z]),
                             Q=np.eye(3), axes=np.full(3, 0.1))
            for i in range(6) for j in range(6) for z in (-0.45, 0.45)]
    lo, hi = np.array([-2.0, -2.0, -1.0]), np.array([2.0, 2.0, 1.0])
    return scenes.Scene(name="many", cfg=0, frame=0, cams=rig, masks=scenes.render_masks(rig, ells),
                        ellipsoids=ells, vol_lo=lo, vol_hi=hi, origin=lo.astype(np.float32),
                        hc_um=62500, hf_um=20000, coarse_dims=(64, 64, 32))


def test_frame_with_more_rois_than_a_wave(fvv, ctx):
    sc = many_balls_scene()
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims, sc.t_np,
                       sc.t_nb, sc.n_steps)
    assert len(res.rois) == 72
    _, bufs, _ = run_frame(fvv, ctx, sc)
    assert ctx.check() == fvv.FVV_OK
    compare_frame(fvv, sc, bufs, res)
    # fewer ROI slots than components: the first ones carried, the flag set
    _, bufs, _ = run_frame(fvv, ctx, sc, max_rois=60)
    counts = host(bufs.counts)
    assert int(counts[0]) == 72 and int(counts[3]) == 60
    jobs = bufs.jobs_host(60)
    for t in range(60):
        assert tuple(jobs[t]["lo"]) == res.fine[t].lo and tuple(jobs[t]["dims"]) == res.fine[t].dims
    assert ctx.check() == fvv.FVV_ECAPACITY
    # fine room for 66 ROIs: the layout stops inside its second run of 64
    sizes = [l.size for l in res.fine]
    _, bufs, _ = run_frame(fvv, ctx, sc, max_fine=sum(sizes[:66]) + sizes[66] // 2)
    counts = host(bufs.counts)
    assert int(counts[0]) == 72 and int(counts[3]) == 66
    assert int(counts[1]) == sum(sizes[:66])
    jobs = bufs.jobs_host(66)
    for t in range(66):
        assert tuple(jobs[t]["lo"]) == res.fine[t].lo and tuple(jobs[t]["dims"]) == res.fine[t].dims
        assert int(jobs[t]["out_offset"]) == sum(sizes[:t])
    assert ctx.check() == fvv.FVV_ECAPACITY


_frame_oracle = {}


def oracle_frame(sc, cfg, frame):
    key = (cfg, frame)
    if key not in _frame_oracle:
        _frame_oracle[key] = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um,
                                          sc.coarse_dims, sc.t_np, sc.t_nb, sc.n_steps)
    return _frame_oracle[key]


# coarse tiles of 32 and 16 samples in x OR their bits into shared bitmap
# words; fine tiles of depth 4 take the culled carve at every width, other
# depths the batched carve
@pytest.mark.parametrize("cfg,frame,ct,ft", [
    (1, 0, (32, 2), (32, 4)), (1, 1, (16, 1), (16, 4)), (1, 2, (64, 2), (64, 2)),
    (1, 0, (16, 4), (32, 8)), (2, 0, (32, 1), (16, 4)), (2, 1, (64, 1), (32, 4))])
def test_frame_tile_shapes(fvv, ctx, scene_cache, cfg, frame, ct, ft):
    sc = scene_cache(cfg, frame)
    res = oracle_frame(sc, cfg, frame)
    _, bufs, _ = run_frame(fvv, ctx, sc, coarse_tile=fvv.tile(*ct), fine_tile=fvv.tile(*ft))
    assert ctx.check() == fvv.FVV_OK
    compare_frame(fvv, sc, bufs, res)


def test_frame_dense_coarse_hull(fvv, ctx, scene_cache):
    """All-foreground silhouettes: every coarse sample is occupied, far more
    than one workgroup's LDS forest holds, so the frame labels in global memory."""
    import copy
    sc = copy.copy(scene_cache(1, 0))
    sc.masks = np.ones_like(sc.masks)
    sc.masks[0, :, 150:154] = 0                # a thin empty band: two halves, crossing edges
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims, sc.t_np,
                       sc.t_nb, sc.n_steps)
    assert res.occ_coarse.sum() > 10000
    _, bufs, _ = run_frame(fvv, ctx, sc)
    assert ctx.check() == fvv.FVV_OK
    compare_frame(fvv, sc, bufs, res)


@pytest.mark.parametrize("cfg", [2, 3])
def test_frame_graph_replays(fvv, ctx, scene_cache, cfg):
    """Replays of a captured frame, eager work between them; the judo frame's
    coarse lattice (18900 tiles) takes the two-pass coarse carve, whose tile
    count the labelling and whose block bits the second pass clear again."""
    import torch
    sc = scene_cache(cfg, 0)
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims)
    g, bufs, sils = run_frame(fvv, ctx, sc, graph=True)
    for rep in range(4):
        for t in (bufs.occ_fine, bufs.keys, bufs.xyz, bufs.labels, bufs.counts):
            t.fill_(0 if rep % 2 else 3)
        g.launch()
        torch.cuda.synchronize()
        x = torch.randn(1000, device="cuda").sum()          # eager work between replays
        torch.cuda.synchronize()
        compare_frame(fvv, sc, bufs, res)
    g.close()
    assert ctx.check() == fvv.FVV_OK


def test_frame_capacity_limits(fvv, ctx, scene_cache):
    sc = scene_cache(2, 0)
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims)
    sizes = [l.size for l in res.fine]
    cap = sum(sizes[:3]) + sizes[3] // 2              # room for three ROIs only
    _, bufs, _ = run_frame(fvv, ctx, sc, max_fine=cap)
    counts = host(bufs.counts)
    assert int(counts[0]) == len(res.rois) and int(counts[3]) == 3
    assert int(counts[1]) == sum(sizes[:3])
    assert ctx.check() == fvv.FVV_ECAPACITY
    _, bufs, _ = run_frame(fvv, ctx, sc, max_rois=5)
    counts = host(bufs.counts)
    assert int(counts[0]) == len(res.rois) and int(counts[3]) == 5
    assert ctx.check() == fvv.FVV_ECAPACITY


def test_invalid_arguments_are_rejected(fvv, ctx, scene_cache):
    sc = scene_cache(1, 0)
    sils = sils_dev(ctx, sc.masks)
    bad = [
        fvv.Grid(origin=(0, 0, 0), h=0.1, lo=(0, 0, 0), dims=(0, 4, 4)),
        fvv.Grid(origin=(0, 0, 0), h=-0.1, lo=(0, 0, 0), dims=(4, 4, 4)),
        fvv.Grid(origin=(0, 0, 0), h=0.1, lo=(1 << 24, 0, 0), dims=(4, 4, 4)),
        fvv.Grid(origin=(0, 0, 0), h=0.1, lo=(0, 0, 0), dims=(1 << 16, 1 << 16, 1)),
    ]
    for g in bad:
        with pytest.raises(fvv.FvvError) as e:
            ctx.carve(sc.P32, sc.W, sc.H, sils, g, out=dev(np.zeros(1, np.uint8)))
        assert e.value.status == fvv.FVV_EINVAL
    good = fvv.Grid(origin=(0, 0, 0), h=0.1, lo=(0, 0, 0), dims=(4, 4, 4))
    P = sc.P32.copy()
    P[1, 0, 0] = np.nan
    with pytest.raises(fvv.FvvError):
        ctx.carve(P, sc.W, sc.H, sils, good)
    with pytest.raises(fvv.FvvError):
        ctx.carve(np.zeros((33, 3, 4), np.float32), sc.W, sc.H, sils, good)
    with pytest.raises(fvv.FvvError):
        ctx.surface(good, dev(np.zeros((4, 4, 4), np.uint8)), sc.P32, sc.W, sc.H, sils, n_steps=13)
    with pytest.raises(fvv.FvvError):
        ctx.label(good, dev(np.zeros((4, 4, 4), np.uint8)), t_np=9, t_nb=8)


@pytest.mark.parametrize("idx", [[0, 8, 16], list(range(17)), list(range(24)) + list(range(8))],
                         ids=["3cams", "17cams", "32cams"])
def test_frame_two_pass_camera_counts(fvv, ctx, scene_cache, idx):
    """The judo frame seen by 3, 17 and 32 cameras (the last repeating 8 of its
    24): the two-pass coarse carve's rejection pass with its box count per
    workgroup capped by the wave (64 boxes of 3 cameras), uneven (15 boxes of 17
    cameras) and at the camera limit (8 boxes of 32; two 16-camera groups per
    kept box), against the oracle."""
    import copy
    sc = copy.copy(scene_cache(3, 0))
    sc.masks = sc.masks[idx]
    sc.cams = [sc.cams[i] for i in idx]
    assert int(np.prod(sc.coarse_dims)) >= 1 << 21
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims, sc.t_np,
                       sc.t_nb, sc.n_steps)
    _, bufs, _ = run_frame(fvv, ctx, sc)
    assert ctx.check() == fvv.FVV_OK
    compare_frame(fvv, sc, bufs, res)


def test_frame_two_pass_empty_and_refilled(fvv, ctx, scene_cache):
    """The two-pass coarse carve with nothing to keep (all-background silhouettes:
    every box rejected, no ROI), then the same context on the real frame (the
    kept-box count and the block bits cleared in between), both against the
    oracle."""
    import copy
    sc0 = scene_cache(3, 0)
    empty = copy.copy(sc0)
    empty.masks = np.zeros_like(sc0.masks)
    for sc in (empty, sc0):
        res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims,
                           sc.t_np, sc.t_nb, sc.n_steps)
        _, bufs, _ = run_frame(fvv, ctx, sc)
        assert ctx.check() == fvv.FVV_OK
        compare_frame(fvv, sc, bufs, res)
        if sc is empty:
            assert len(res.rois) == 0 and int(host(bufs.occ_coarse).sum()) == 0


# ------------------------------------------------------------------ paper-shaped frames
@pytest.mark.parametrize("cfg", [scenes.CFG_PAPER_V, scenes.CFG_JUDO_FINE])
def test_frame_paper_shapes(fvv, scene_cache, cfg):
    """The paper's volleyball shape (10 cameras 3840x2160, an 18 x 18 x 9 m volume at
    50 mm: 360 x 360 x 180 coarse samples, carved in two passes; 20 mm fine) and a
    judo frame at 2 mm (~1.9e8 fine samples in 6 ROIs, fine bitmaps and job tables
    at that size) against the oracle, element by element."""
    sc = scene_cache(cfg, 0)
    res = oracle_frame(sc, cfg, 0)
    c = fvv.Context(max_cams=sc.P32.shape[0], max_w=sc.W, max_h=sc.H,
                    max_coarse=int(np.prod(sc.coarse_dims)), max_fine=1 << 28, max_rois=256,
                    max_points=1 << 22, max_jobs=256)
    try:
        _, bufs, _ = run_frame(fvv, c, sc, max_rois=256, max_fine=1 << 28, max_points=1 << 22)
        assert c.check() == fvv.FVV_OK
        compare_frame(fvv, sc, bufs, res)
        if cfg == scenes.CFG_JUDO_FINE:
            assert res.fine_voxels > 100_000_000
    finally:
        c.close()
