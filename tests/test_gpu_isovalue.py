"""GPU parity of the paper's Bresenham isovalue (fvv_isovalue) against the
oracle (oracle.isovalue).  lambda is a correctly rounded function of integers
(the double quotient of two squared pixel lengths, its minimum over cameras,
the square root rounded to float), and the point is one fp32 add and one fma
from it, so both are compared bit for bit: on the tiny scene's ROIs with the
keys of fvv_surface, a volleyball and a judo frame's ROIs as fvv_frame leaves
them, a ball seen with ~7 px edges (longer walks), keys that name no edge,
key counts past max_keys, a camera behind the lattice, and invalid
arguments."""
import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fvv():
    import paper_1903_11785_amd as fvv
    return fvv


@pytest.fixture(scope="module")
def ctx(fvv):
    c = fvv.Context(max_coarse=5_000_000, max_fine=1 << 26, max_rois=256, max_points=1 << 22,
                    max_jobs=256)
    yield c
    c.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def grid_of(fvv, lat):
    return fvv.Grid(origin=tuple(np.float32(lat.origin)), h=np.float32(lat.h), lo=tuple(lat.lo),
                    dims=tuple(lat.dims))


def gpu_iso(fvv, ctx, lat, occ, P, W, H, sils_dev, keys, n=None, max_keys=None):
    import torch
    k = dev(keys.astype(np.uint32).view(np.int32) if keys.size else np.zeros(1, np.int32))
    if max_keys is not None:
        k = k[:max_keys]
    nk = torch.tensor([keys.size if n is None else n], dtype=torch.int32, device="cuda")
    lam, xyz = ctx.isovalue(grid_of(fvv, lat), dev(occ), P, W, H, sils_dev, k, nk)
    return lam.cpu().numpy(), xyz.cpu().numpy()


def assert_same(lam, xyz, ref_lam, ref_xyz):
    np.testing.assert_array_equal(lam.view(np.uint32), ref_lam.view(np.uint32))
    np.testing.assert_array_equal(xyz.view(np.uint32), ref_xyz.view(np.uint32))


def test_tiny_scene_rois(fvv, ctx, scene_cache):
    for frame in (0, 1, 2):
        sc = scene_cache(scenes.CFG_TINY, frame)
        res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims,
                           sc.t_np, sc.t_nb, sc.n_steps)
        sils = ctx.pack_silhouettes(dev(sc.masks))
        hs = oracle.pack(sc.masks)
        for lat, occ, keys in zip(res.fine, res.occ_fine, res.keys):
            # keys as fvv_surface leaves them, on the device
            g = grid_of(fvv, lat)
            occ_d = dev(occ)
            kd, _, nd = ctx.surface(g, occ_d, sc.P32, sc.W, sc.H, sils, n_steps=sc.n_steps)
            lam, xyz = ctx.isovalue(g, occ_d, sc.P32, sc.W, sc.H, sils, kd, nd)
            n = int(nd.cpu()[0])
            ref_lam, ref_xyz = oracle.isovalue(sc.P32, hs, sc.W, sc.H, lat, occ, keys)
            assert n == keys.size
            assert_same(lam[:n].cpu().numpy(), xyz[:n].cpu().numpy(), ref_lam, ref_xyz)
    assert ctx.check() == fvv.FVV_OK


@pytest.mark.parametrize("cfg", [scenes.CFG_VOLLEYBALL, scenes.CFG_JUDO])
def test_frame_rois(fvv, ctx, scene_cache, cfg):
    """Every second ROI of a full-size frame, on the frame's own fine
    occupancy and keys (the launch shape a frame would use)."""
    import torch
    sc = scene_cache(cfg, 0)
    coarse = fvv.Grid(origin=tuple(sc.origin), h=sc.hc, lo=(0, 0, 0), dims=sc.coarse_dims)
    params = fvv.frame_params(sc.P32, sc.W, sc.H, coarse, sc.hc_um, sc.hf_um, sc.t_np, sc.t_nb,
                              sc.n_steps)
    bufs = fvv.FrameBuffers(coarse, 256, 1 << 26, 1 << 22)
    N, H, W = sc.masks.shape
    sils = torch.zeros((N, H, (W + 31) // 32), dtype=torch.int32, device="cuda")
    ctx.frame(params, sils, bufs, masks=dev(sc.masks))
    torch.cuda.synchronize()
    assert ctx.check() == fvv.FVV_OK
    K = int(bufs.counts.cpu()[0])
    jobs = bufs.jobs_host(K)
    poff = bufs.point_off.cpu().numpy().view(np.uint32)
    hs = sils.cpu().numpy().view(np.uint32)
    total = 0
    for t in range(0, K, 2):
        g = jobs[t]
        dims = tuple(int(v) for v in g["dims"])
        lat = oracle.Lattice(origin=np.asarray(g["origin"], np.float32), h=np.float32(g["h"]),
                             lo=tuple(int(v) for v in g["lo"]), dims=dims)
        o = int(g["out_offset"])
        occ_d = bufs.occ_fine[o:o + int(np.prod(dims))]
        kd = bufs.keys[int(poff[t]):int(poff[t + 1])]
        nd = torch.tensor([kd.numel()], dtype=torch.int32, device="cuda")
        lam, xyz = ctx.isovalue(grid_of(fvv, lat), occ_d, sc.P32, sc.W, sc.H, sils, kd, nd)
        occ = occ_d.cpu().numpy().reshape(dims[2], dims[1], dims[0])
        keys = kd.cpu().numpy().view(np.uint32)
        ref_lam, ref_xyz = oracle.isovalue(sc.P32, hs, sc.W, sc.H, lat, occ, keys)
        assert_same(lam.cpu().numpy(), xyz.cpu().numpy(), ref_lam, ref_xyz)
        total += keys.size
    assert total > 10000


def test_ball_with_long_edges(fvv, ctx):
    from test_oracle_isovalue import ball_scene
    sc, lat = ball_scene()
    hs = oracle.pack(sc.masks)
    occ, _ = oracle.carve(sc.P32, hs, sc.W, sc.H, lat)
    keys = oracle.edges(occ)
    lam, xyz = gpu_iso(fvv, ctx, lat, occ, sc.P32, sc.W, sc.H, dev(hs.view(np.int32)), keys)
    ref_lam, ref_xyz = oracle.isovalue(sc.P32, hs, sc.W, sc.H, lat, occ, keys)
    assert_same(lam, xyz, ref_lam, ref_xyz)
    assert (ref_lam > 0).mean() > 0.5          # walks of several pixels


def test_keys_that_name_no_edge_and_counts(fvv, ctx, scene_cache):
    sc = scene_cache(scenes.CFG_TINY, 0)
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims)
    lat, occ, keys = res.fine[0], res.occ_fine[0], res.keys[0]
    hs = oracle.pack(sc.masks)
    sils = dev(hs.view(np.int32))
    nx, ny, nz = lat.dims
    bad = np.array([3 * (nx - 1) + 0,                      # x-edge leaving the lattice
                    3 * (nx * (ny - 1)) + 1,               # y-edge leaving it
                    3 * (nx * ny * (nz - 1)) + 2,          # z-edge leaving it
                    3 * (nx * ny * nz) + 0], np.uint32)    # past the last sample
    mixed = np.concatenate([keys[:5], bad, keys[5:9]])
    lam, xyz = gpu_iso(fvv, ctx, lat, occ, sc.P32, sc.W, sc.H, sils, mixed)
    ref_lam, ref_xyz = oracle.isovalue(sc.P32, hs, sc.W, sc.H, lat, occ, keys[:9])
    assert np.isnan(lam[5:9]).all() and np.isnan(xyz[5:9]).all()
    assert_same(np.concatenate([lam[:5], lam[9:]]), np.concatenate([xyz[:5], xyz[9:]]),
                ref_lam, ref_xyz)
    # *n_keys past max_keys: the first max_keys are done, the rest untouched
    import torch
    k = dev(keys[:20].view(np.int32))
    nk = torch.tensor([1000], dtype=torch.int32, device="cuda")
    lam_d = torch.full((20,), -5.0, device="cuda")
    lam2, _ = ctx.isovalue(grid_of(fvv, lat), dev(occ), sc.P32, sc.W, sc.H, sils, k[:12], nk,
                           lam=lam_d)
    got = lam_d.cpu().numpy()
    ref20, _ = oracle.isovalue(sc.P32, hs, sc.W, sc.H, lat, occ, keys[:12])
    np.testing.assert_array_equal(got[:12].view(np.uint32), ref20.view(np.uint32))
    # zero keys: nothing written
    nk0 = torch.zeros(1, dtype=torch.int32, device="cuda")
    lam_d.fill_(-5.0)
    ctx.isovalue(grid_of(fvv, lat), dev(occ), sc.P32, sc.W, sc.H, sils, k, nk0, lam=lam_d)
    assert (lam_d.cpu().numpy() == -5.0).all()
    assert ctx.check() == fvv.FVV_OK


def test_camera_behind_the_lattice(fvv, ctx, scene_cache):
    """A fifth camera facing away: both sides give lambda_i = 0 for it, so
    every lambda is 0 (the oracle's reading of a camera behind the edge)."""
    sc = scene_cache(scenes.CFG_TINY, 0)
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims)
    lat, occ, keys = res.fine[0], res.occ_fine[0], res.keys[0]
    P = np.concatenate([sc.P32, -sc.P32[:1]], 0)           # w < 0 for every sample
    masks = np.concatenate([sc.masks, np.ones_like(sc.masks[:1])], 0)
    hs = oracle.pack(masks)
    lam, xyz = gpu_iso(fvv, ctx, lat, occ, P, sc.W, sc.H, dev(hs.view(np.int32)), keys)
    ref_lam, ref_xyz = oracle.isovalue(P, hs, sc.W, sc.H, lat, occ, keys)
    assert_same(lam, xyz, ref_lam, ref_xyz)
    assert (ref_lam == 0).all()


def test_invalid_isovalue_arguments(fvv, ctx, scene_cache):
    import torch
    sc = scene_cache(scenes.CFG_TINY, 0)
    occ = torch.zeros((4, 4, 4), dtype=torch.uint8, device="cuda")
    sils = ctx.pack_silhouettes(dev(sc.masks))
    keys = torch.zeros(4, dtype=torch.int32, device="cuda")
    nk = torch.zeros(1, dtype=torch.int32, device="cuda")
    good = fvv.Grid(origin=(0.0, 0.0, 0.0), h=np.float32(0.01), lo=(0, 0, 0), dims=(4, 4, 4))
    bad_dims = fvv.Grid(origin=(0.0, 0.0, 0.0), h=np.float32(0.01), lo=(0, 0, 0), dims=(0, 4, 4))
    huge = fvv.Grid(origin=(0.0, 0.0, 0.0), h=np.float32(0.01), lo=(0, 0, 0),
                    dims=(2048, 2048, 512))
    for g in (bad_dims, huge):
        with pytest.raises(fvv.FvvError) as e:
            ctx.isovalue(g, occ, sc.P32, sc.W, sc.H, sils, keys, nk)
        assert e.value.status == fvv.FVV_EINVAL
    with pytest.raises(fvv.FvvError) as e:
        ctx.isovalue(good, occ, sc.P32[:0], sc.W, sc.H, sils, keys, nk)      # no camera
    assert e.value.status == fvv.FVV_EINVAL


@pytest.mark.parametrize("cfg,frame,graph", [(scenes.CFG_TINY, 0, False), (scenes.CFG_TINY, 1, True),
                                             (scenes.CFG_VOLLEYBALL, 0, False),
                                             (scenes.CFG_VOLLEYBALL, 1, True),
                                             (scenes.CFG_JUDO, 0, False)])
def test_frame_with_the_bresenham_estimator(fvv, ctx, scene_cache, cfg, frame, graph):
    """fvv_frame with exit_estimator = EXIT_BRESENHAM: every exit point equals
    the oracle's isovalue point on the oracle's own fine occupancy and keys
    (one launch over all ROIs in place of the bisection); as a graph, on
    every replay."""
    import torch
    sc = scene_cache(cfg, frame)
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims, sc.t_np,
                       sc.t_nb, sc.n_steps)
    hs = oracle.pack(sc.masks)
    ref = [oracle.isovalue(sc.P32, hs, sc.W, sc.H, lat, occ, keys)[1]
           for lat, occ, keys in zip(res.fine, res.occ_fine, res.keys)]
    coarse = fvv.Grid(origin=tuple(sc.origin), h=sc.hc, lo=(0, 0, 0), dims=sc.coarse_dims)
    params = fvv.frame_params(sc.P32, sc.W, sc.H, coarse, sc.hc_um, sc.hf_um, sc.t_np, sc.t_nb,
                              sc.n_steps, exit_estimator=fvv.EXIT_BRESENHAM)
    bufs = fvv.FrameBuffers(coarse, 256, 1 << 26, 1 << 22)
    N, H, W = sc.masks.shape
    sils = torch.zeros((N, H, (W + 31) // 32), dtype=torch.int32, device="cuda")
    masks = dev(sc.masks)
    runs = 3 if graph else 1
    g = ctx.frame_graph(params, sils, bufs, masks=masks) if graph else None
    for _ in range(runs):
        bufs.xyz.fill_(-1.0)
        torch.cuda.synchronize()
        if graph:
            g.launch()
        else:
            ctx.frame(params, sils, bufs, masks=masks)
        torch.cuda.synchronize()
        assert ctx.check() == fvv.FVV_OK
        poff = bufs.point_off.cpu().numpy().view(np.uint32)
        xyz = bufs.xyz.cpu().numpy()
        assert int(bufs.counts.cpu()[3]) == len(ref)
        for t, r in enumerate(ref):
            got = xyz[poff[t]:poff[t + 1]]
            np.testing.assert_array_equal(got.view(np.uint32), r.view(np.uint32))
    if g is not None:
        g.close()


def test_frame_rejects_an_unknown_estimator(fvv, ctx, scene_cache):
    import torch
    sc = scene_cache(scenes.CFG_TINY, 0)
    coarse = fvv.Grid(origin=tuple(sc.origin), h=sc.hc, lo=(0, 0, 0), dims=sc.coarse_dims)
    params = fvv.frame_params(sc.P32, sc.W, sc.H, coarse, sc.hc_um, sc.hf_um, exit_estimator=2)
    bufs = fvv.FrameBuffers(coarse, 16, 1 << 22, 1 << 16)
    N, H, W = sc.masks.shape
    sils = torch.zeros((N, H, (W + 31) // 32), dtype=torch.int32, device="cuda")
    with pytest.raises(fvv.FvvError) as e:
        ctx.frame(params, sils, bufs, masks=dev(sc.masks))
    assert e.value.status == fvv.FVV_EINVAL
