"""GPU parity of the depth images and visibility (fvv_visibility) against the
oracle (oracle.depth, oracle.visibility).  Both evaluate the same fp32
operations in the same order with IEEE division, and the minimum of Eq. (4)
does not depend on the order of the updates, so depth images and masks are
compared bit for bit: the pins' hand-built triangles, a closed sphere mesh in
three cameras, and the full mesh of a volleyball frame (its exit points and
triangles as fvv_frame leaves them) in its 16 cameras at 1920x1080; counts
past the capacities, missing vertices, and invalid arguments."""
import numpy as np
import pytest

import oracle
import scenes
from test_oracle_visibility import cam_P, sphere_mesh, tri_at, two_triangles, W, H

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


def gpu_vis(ctx, P, Wd, Hd, xyz, tris, t_v, n_vert=None, n_tris=None):
    import torch
    nv = torch.tensor([xyz.shape[0] if n_vert is None else n_vert], dtype=torch.int32,
                      device="cuda")
    nt = torch.tensor([tris.shape[0] if n_tris is None else n_tris], dtype=torch.int32,
                      device="cuda")
    D, vis = ctx.visibility(P, Wd, Hd, dev(xyz.astype(np.float32)), nv,
                            dev(tris.astype(np.uint32).view(np.int32)), nt, t_v)
    return D.cpu().numpy(), vis.cpu().numpy().view(np.uint32)


def check(P, Wd, Hd, xyz, tris, t_v, D, vis):
    rD = oracle.depth(P, Wd, Hd, xyz, tris)
    rv = oracle.visibility(P, Wd, Hd, xyz, tris, rD, t_v)
    np.testing.assert_array_equal(D.view(np.uint32), rD.view(np.uint32))
    np.testing.assert_array_equal(vis, rv)
    return rD, rv


@pytest.mark.parametrize("t_v", [0.5, 1.5])
def test_hand_built_triangles(fvv, ctx, t_v):
    P = cam_P()
    xyz, tris = two_triangles()
    extra = np.concatenate([
        tri_at([(10.3, 12.7), (50.6, 20.1), (25.2, 55.9)], 2.5),
        tri_at([(70.5, 5.5), (90.5, 8.5), (80.5, 30.5)], 2.0),                 # outside
        tri_at([(10.5, 10.5), (30.5, 10.5), (20.5, 30.5)], 2.0) * np.float32([1, 1, -1]),
        tri_at([(10.5, 10.5), (20.5, 20.5), (30.5, 30.5)], 2.0)])              # collinear
    xyz = np.concatenate([xyz, extra])
    tris = np.concatenate([tris, np.arange(6, 18, dtype=np.uint32).reshape(4, 3),
                           np.array([[0, 1, 0xffffffff]], np.uint32)])
    D, vis = gpu_vis(ctx, P, W, H, xyz, tris, t_v)
    check(P, W, H, xyz, tris, t_v, D, vis)


def test_sphere(fvv, ctx):
    xyz, tris = sphere_mesh()
    cams = [scenes.look_at(np.array(c) * 1.5, np.zeros(3), 300.0, 200, 200)
            for c in [(1.0, 0.2, 0.3), (-0.3, 1.0, 0.1), (0.1, -0.4, 1.0)]]
    P = np.stack([c.P32 for c in cams])
    D, vis = gpu_vis(ctx, P, 200, 200, xyz, tris, 0.025)
    rD, rv = check(P, 200, 200, xyz, tris, 0.025, D, vis)
    assert np.isfinite(rD).sum() > 15000 and 0.3 < np.mean(rv & 1) < 0.7


def test_volleyball_frame_mesh(fvv, ctx, scene_cache):
    """The mesh of a volleyball frame (exit points, triangles with frame-wide
    vertex indices) in its 16 cameras at 1920x1080, T_v = 0.1 m."""
    import torch
    sc = scene_cache(scenes.CFG_VOLLEYBALL, 0)
    coarse = fvv.Grid(origin=tuple(sc.origin), h=sc.hc, lo=(0, 0, 0), dims=sc.coarse_dims)
    params = fvv.frame_params(sc.P32, sc.W, sc.H, coarse, sc.hc_um, sc.hf_um, sc.t_np, sc.t_nb,
                              sc.n_steps)
    bufs = fvv.FrameBuffers(coarse, 256, 1 << 26, 1 << 22, max_tris=1 << 21)
    N, Hh, Ww = sc.masks.shape
    sils = torch.zeros((N, Hh, (Ww + 31) // 32), dtype=torch.int32, device="cuda")
    ctx.frame(params, sils, bufs, masks=dev(sc.masks))
    torch.cuda.synchronize()
    assert ctx.check() == fvv.FVV_OK
    K = int(bufs.counts.cpu()[0])
    n_t = bufs.tri_off[K:K + 1]
    n_p = bufs.counts[2:3]
    D, vis = ctx.visibility(sc.P32, sc.W, sc.H, bufs.xyz, n_p, bufs.tris, n_t, 0.1)
    T = int(n_t.cpu()[0])
    E = int(n_p.cpu()[0])
    xyz = bufs.xyz[:E].cpu().numpy()
    tris = bufs.tris[:T].cpu().numpy().view(np.uint32)
    assert T > 100000
    rD, rv = check(sc.P32, sc.W, sc.H, xyz, tris, 0.1, D.cpu().numpy(),
                   vis[:T].cpu().numpy().view(np.uint32))
    # players occlude each other in some cameras; most triangles are seen by several
    seen = np.array([bin(int(v)).count("1") for v in rv[::97]])
    assert seen.mean() > 4


def test_counts_past_capacity(fvv, ctx):
    import torch
    xyz, tris = sphere_mesh()
    cams = [scenes.look_at(np.array([1.0, 0.2, 0.3]) * 1.5, np.zeros(3), 300.0, 200, 200)]
    P = np.stack([c.P32 for c in cams])
    T = tris.shape[0]
    # *n_tris above the capacity: the first max_tris triangles
    D, vis = gpu_vis(ctx, P, 200, 200, xyz, tris[:T // 2], 0.025, n_tris=T)
    check(P, 200, 200, xyz, tris[:T // 2], 0.025, D, vis)
    # fewer vertices than the triangles name: those triangles are skipped
    nv = xyz.shape[0] // 2
    D, vis = gpu_vis(ctx, P, 200, 200, xyz, tris, 0.025, n_vert=nv)
    check(P, 200, 200, xyz[:nv], tris, 0.025, D, vis)
    # zero triangles: the depth images are all +inf
    D, vis = gpu_vis(ctx, P, 200, 200, xyz, tris[:4], 0.025, n_tris=0)
    assert np.isinf(D).all()


def test_invalid_visibility_arguments(fvv, ctx):
    import torch
    xyz = torch.zeros((4, 3), device="cuda")
    tris = torch.zeros((2, 3), dtype=torch.int32, device="cuda")
    n = torch.ones(1, dtype=torch.int32, device="cuda")
    P = cam_P()
    for t_v in (float("nan"), float("inf")):
        with pytest.raises(fvv.FvvError) as e:
            ctx.visibility(P, W, H, xyz, n, tris, n, t_v)
        assert e.value.status == fvv.FVV_EINVAL
    with pytest.raises(fvv.FvvError) as e:
        ctx.visibility(P[:0], W, H, xyz, n, tris, n, 0.1)
    assert e.value.status == fvv.FVV_EINVAL
