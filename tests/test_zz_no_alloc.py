"""fvv_surface_noalloc (the exit-point pass of one ROI with the library's static
per-GPU scratch, for callers that cannot allocate) against fvv_surface through
the C ABI: keys and point counts bit-exact, exit points within 1e-4 of the
voxel edge, on two calls in a row, the second on a smaller lattice, and both
against the oracle's crossing edges and bisection (Sec. II-C)."""
import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _grid(fvv, lat):
    return fvv.Grid(origin=tuple(np.float32(lat.origin)), h=np.float32(lat.h), lo=tuple(lat.lo),
                    dims=tuple(lat.dims))


def _call_both(fvv, ctx, sc, lat, occ, sils, max_points):
    import torch
    keys_a, xyz_a, n_a = ctx.surface(_grid(fvv, lat), _dev(occ), sc.P32, sc.W, sc.H, sils, 8,
                                     max_points)
    keys_b = torch.full((max_points,), -7, dtype=torch.int32, device="cuda")
    xyz_b = torch.full((max_points, 3), 7.0, dtype=torch.float32, device="cuda")
    n_b = torch.zeros(1, dtype=torch.int32, device="cuda")
    fvv.surface_noalloc(_grid(fvv, lat), _dev(occ), sc.P32, sc.W, sc.H, sils, keys_b, xyz_b, n_b,
                        n_steps=8, max_points=max_points)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (keys_a, xyz_a, n_a, keys_b, xyz_b, n_b)]


def test_noalloc_surface_equals_surface_twice(scene_cache):
    import paper_1903_11785_amd as fvv
    sc = scene_cache(scenes.CFG_TINY, 0)
    res = oracle.frame(sc.masks, sc.P32, sc.origin, sc.hc_um, sc.hf_um, sc.coarse_dims,
                       surface=False)
    big = int(np.argmax([lat.size for lat in res.fine]))
    lat1, occ1 = res.fine[big], res.occ_fine[big]
    # the second call: a smaller lattice, a sub-box of the first at an offset
    nx, ny, nz = lat1.dims
    sub = (max(nx // 2, 1), max(ny // 2, 1), max(nz // 2, 1))
    off = (nx // 4, ny // 3, nz // 5)
    lat2 = oracle.Lattice(origin=lat1.origin, h=lat1.h,
                          lo=tuple(l + o for l, o in zip(lat1.lo, off)), dims=sub)
    occ2 = np.ascontiguousarray(occ1[off[2]:off[2] + sub[2], off[1]:off[1] + sub[1],
                                     off[0]:off[0] + sub[0]])
    assert lat2.size < lat1.size
    ctx = fvv.Context(max_coarse=1 << 20, max_fine=1 << 24, max_rois=64, max_points=1 << 20)
    try:
        sils = ctx.pack_silhouettes(_dev(sc.masks))
        packed = oracle.pack(sc.masks)
        for lat, occ in ((lat1, occ1), (lat2, occ2)):
            ka, xa, na, kb, xb, nb = _call_both(fvv, ctx, sc, lat, occ, sils, 1 << 20)
            keys_ref = oracle.edges(occ)
            xyz_ref, _ = oracle.bisect(sc.P32, packed, sc.W, sc.H, lat, occ, keys_ref, 8)
            E = int(na[0])
            assert E == int(nb[0]) == keys_ref.size > 0
            np.testing.assert_array_equal(kb[:E], ka[:E])
            np.testing.assert_array_equal(kb[:E].view(np.uint32), keys_ref)
            assert (kb[E:] == -7).all() and (xb[E:] == 7.0).all()
            tol = 1e-4 * float(lat.h)
            assert np.abs(xb[:E].astype(np.float64) - xa[:E]).max() <= tol
            assert np.abs(xb[:E].astype(np.float64) - xyz_ref).max() <= tol
        # capacity: the count is complete, only the first max_points written
        ka, xa, na, kb, xb, nb = _call_both(fvv, ctx, sc, lat1, occ1, sils, 1000)
        assert int(nb[0]) == int(na[0]) > 1000
        np.testing.assert_array_equal(kb, ka)
        assert np.abs(xb.astype(np.float64) - xa).max() <= 1e-4 * float(lat1.h)
        assert ctx.check() == fvv.FVV_ECAPACITY
    finally:
        ctx.close()


def test_noalloc_surface_rejects_lattices_past_its_scratch(scene_cache):
    import torch
    import paper_1903_11785_amd as fvv
    sc = scene_cache(scenes.CFG_TINY, 0)
    keys = torch.zeros(16, dtype=torch.int32, device="cuda")
    xyz = torch.zeros((16, 3), dtype=torch.float32, device="cuda")
    n = torch.zeros(1, dtype=torch.int32, device="cuda")
    sils = torch.zeros((4, sc.H, (sc.W + 31) // 32), dtype=torch.int32, device="cuda")
    occ = torch.zeros(1, dtype=torch.uint8, device="cuda")
    # ny * nz rows of one word each: one row past the limit
    too_big = fvv.Grid(origin=(0.0, 0.0, 0.0), h=0.01, lo=(0, 0, 0),
                       dims=(64, 1024, fvv.NOALLOC_BITMAP_WORDS // 1024 + 1))
    with pytest.raises(fvv.FvvError) as e:
        fvv.surface_noalloc(too_big, occ, sc.P32, sc.W, sc.H, sils, keys, xyz, n)
    assert e.value.status == fvv.FVV_EINVAL
    with pytest.raises(fvv.FvvError):
        fvv.surface_noalloc(too_big, occ, sc.P32, sc.W, sc.H, sils, keys, xyz, n, n_steps=13)
