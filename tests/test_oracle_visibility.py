"""Pins of the oracle's depth images and visibility (oracle.depth,
oracle.visibility; Sec. II-D, Eq. (4)).

  - a fronto-parallel triangle: the covered pixels are exactly those whose
    centres lie inside it by a double-precision barycentric test (pixels
    within 1e-4 of an edge skipped), at the triangle's depth, +inf elsewhere;
  - two overlapping triangles at depths 2 and 3: the overlap holds 2 (Eq. (4)'s
    minimum), the rest of the far one 3; the far triangle is occluded when its
    centroid's pixel is covered by the near one and T_v is below the gap, and
    visible when T_v exceeds it (self-occlusion ignored), the near one always;
  - triangles outside the image or behind the camera are invisible and leave
    no depth; a zero-area triangle leaves no depth; a triangle naming a
    vertex past the vertex count is skipped;
  - the depth image does not depend on the order of the triangles;
  - a closed sphere mesh seen from outside: triangles well behind the
    sphere's centre (camera-plane distance beyond it by 0.3 r) are occluded,
    those well in front of it (0.5 r) visible, for T_v = 0.1 r (nearer the
    rim, where the surface is steep, a triangle's constant distance can differ
    from its neighbours' by more than T_v: the self-occlusion a high T_v is
    there to ignore).
"""
import numpy as np
import pytest

import oracle
import scenes

F, W, H = 100.0, 64, 64


def cam_P(f=F, cx=W / 2, cy=H / 2):
    """Camera at the origin looking along +z: w = Z."""
    K = np.array([[f, 0, cx], [0, f, cy], [0, 0, 1.0]])
    return (K @ np.hstack([np.eye(3), np.zeros((3, 1))])).astype(np.float32).reshape(1, 12)


def tri_at(pix, Z):
    """World vertices of a triangle at depth Z projecting to pixel coordinates pix."""
    pix = np.asarray(pix, np.float64)
    X = (pix[:, 0] - W / 2) * Z / F
    Y = (pix[:, 1] - H / 2) * Z / F
    return np.stack([X, Y, np.full(3, Z)], 1).astype(np.float32)


def inside_double(P, V, x, y):
    """+1 inside, 0 outside, None within 1e-4 of an edge (barycentric, double)."""
    P = P.reshape(3, 4).astype(np.float64)
    h = np.hstack([V.astype(np.float64), np.ones((3, 1))]) @ P.T
    uv = h[:, :2] / h[:, 2:3]
    A = np.array([[uv[0, 0] - uv[2, 0], uv[1, 0] - uv[2, 0]],
                  [uv[0, 1] - uv[2, 1], uv[1, 1] - uv[2, 1]]])
    l01 = np.linalg.solve(A, np.array([x + 0.5 - uv[2, 0], y + 0.5 - uv[2, 1]]))
    lam = np.array([l01[0], l01[1], 1 - l01.sum()])
    if np.min(np.abs(lam)) < 1e-4:
        return None
    return 1 if (lam > 0).all() else 0


def test_fronto_parallel_triangle_coverage_and_depth():
    P = cam_P()
    V = tri_at([(10.3, 12.7), (50.6, 20.1), (25.2, 55.9)], 2.0)
    D = oracle.depth(P, W, H, V, np.array([[0, 1, 2]], np.uint32))[0]
    checked = 0
    for y in range(H):
        for x in range(W):
            ins = inside_double(P, V, x, y)
            if ins is None:
                continue
            checked += 1
            if ins:
                assert D[y, x] == np.float32(2.0), (x, y)
            else:
                assert np.isinf(D[y, x]), (x, y)
    assert checked > 4000 and np.isfinite(D).sum() > 500
    # the opposite winding covers the same pixels
    D2 = oracle.depth(P, W, H, V, np.array([[0, 2, 1]], np.uint32))[0]
    np.testing.assert_array_equal(D, D2)


def two_triangles():
    near = tri_at([(5.5, 5.5), (60.5, 10.5), (20.5, 58.5)], 2.0)
    far = tri_at([(20.5, 15.5), (58.5, 22.5), (30.5, 60.5)], 3.0)
    xyz = np.concatenate([near, far])
    return xyz, np.array([[0, 1, 2], [3, 4, 5]], np.uint32)


def test_overlap_keeps_the_nearest_distance():
    P = cam_P()
    xyz, tris = two_triangles()
    D = oracle.depth(P, W, H, xyz, tris)[0]
    Dn = oracle.depth(P, W, H, xyz, tris[:1])[0]
    Df = oracle.depth(P, W, H, xyz, tris[1:])[0]
    both = np.isfinite(Dn) & np.isfinite(Df)
    assert both.sum() > 50
    assert (D[both] == 2.0).all()
    assert (D[np.isfinite(Df) & ~np.isfinite(Dn)] == 3.0).all()
    assert (D[np.isfinite(Dn)] == 2.0).all()
    assert np.isinf(D[~np.isfinite(Dn) & ~np.isfinite(Df)]).all()
    # order of the triangles does not matter
    np.testing.assert_array_equal(D, oracle.depth(P, W, H, xyz, tris[::-1].copy())[0])


def test_occlusion_threshold():
    P = cam_P()
    xyz, tris = two_triangles()
    # the far triangle's centroid (~(36.5, 32.8)) lies under the near one
    D = oracle.depth(P, W, H, xyz, tris)
    g = xyz[3:].mean(0)
    u, v = F * g[0] / g[2] + W / 2, F * g[1] / g[2] + H / 2
    covered_by_near = np.isfinite(oracle.depth(P, W, H, xyz, tris[:1])[0][int(v), int(u)])
    vis_low = oracle.visibility(P, W, H, xyz, tris, D, 0.5)
    vis_high = oracle.visibility(P, W, H, xyz, tris, D, 1.5)
    assert vis_low[0] == 1 and vis_high[0] == 1
    assert vis_high[1] == 1
    assert vis_low[1] == (0 if covered_by_near else 1)
    assert covered_by_near                      # the case the layout is built for


def test_out_of_view_behind_and_degenerate():
    P = cam_P()
    outside = tri_at([(70.5, 5.5), (90.5, 8.5), (80.5, 30.5)], 2.0)
    behind = tri_at([(10.5, 10.5), (30.5, 10.5), (20.5, 30.5)], 2.0) * np.float32([1, 1, -1])
    flat = tri_at([(10.5, 10.5), (20.5, 20.5), (30.5, 30.5)], 2.0)      # collinear
    xyz = np.concatenate([outside, behind, flat])
    tris = np.arange(9, dtype=np.uint32).reshape(3, 3)
    D = oracle.depth(P, W, H, xyz, tris)
    assert np.isinf(D).all()
    vis = oracle.visibility(P, W, H, xyz, tris, D, 0.1)
    assert vis[0] == 0 and vis[1] == 0
    # a triangle naming a missing vertex (the mesh writes 0xffffffff) is skipped
    good = tri_at([(10.5, 10.5), (30.5, 12.5), (20.5, 30.5)], 2.0)
    t2 = np.array([[0, 1, 2], [0, 1, 0xffffffff], [3, 1, 2]], np.uint32)
    D2 = oracle.depth(P, W, H, good, t2)
    np.testing.assert_array_equal(D2, oracle.depth(P, W, H, good, t2[:1]))
    vis2 = oracle.visibility(P, W, H, good, t2, D2, 0.1)
    assert vis2.tolist() == [1, 0, 0]


def sphere_mesh(n=28, r=0.25, h=0.02):
    """Marching-cubes triangles of a ball of radius r (edge vertices where the
    sphere cuts the edge), centre at the origin."""
    lat_o = -(n // 2) * h
    g = np.arange(n) * h + lat_o
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    occ = (x * x + y * y + z * z <= r * r).astype(np.uint8)
    keys = oracle.edges(occ)
    tris = oracle.mesh(occ, keys)
    lin, axis = keys // 3, keys % 3
    idx = np.stack([lin % n, (lin // n) % n, lin // (n * n)], 1).astype(np.float64)
    X0 = idx * h + lat_o
    d = np.zeros_like(X0)
    d[np.arange(keys.size), axis] = h
    # root of |X0 + t d| = r on the edge
    a = (d * d).sum(1)
    b = 2 * (X0 * d).sum(1)
    c = (X0 * X0).sum(1) - r * r
    disc = np.sqrt(np.maximum(b * b - 4 * a * c, 0))
    t1, t2 = (-b - disc) / (2 * a), (-b + disc) / (2 * a)
    t = np.where((t1 >= 0) & (t1 <= 1), t1, t2)
    return (X0 + t[:, None] * d).astype(np.float32), tris


def test_sphere_far_side_is_occluded():
    r = 0.25
    xyz, tris = sphere_mesh(r=r)
    cams = [scenes.look_at(np.array(c) * 1.5, np.zeros(3), 300.0, 200, 200)
            for c in [(1.0, 0.2, 0.3), (-0.3, 1.0, 0.1), (0.1, -0.4, 1.0)]]
    P = np.stack([c.P32 for c in cams])
    D = oracle.depth(P, 200, 200, xyz, tris)
    vis = oracle.visibility(P, 200, 200, xyz, tris, D, 0.1 * r)
    G = xyz[tris].astype(np.float64).mean(1)
    for c, cam in enumerate(cams):
        w = (np.hstack([G, np.ones((len(G), 1))]) @ cam.P64.T)[:, 2]
        w_c = (cam.P64 @ np.array([0, 0, 0, 1.0]))[2]
        bit = (vis >> c) & 1
        far = w > w_c + 0.3 * r
        near = w < w_c - 0.5 * r
        assert far.sum() > 100 and near.sum() > 100
        assert (bit[far] == 0).all()
        assert (bit[near] == 1).all()
