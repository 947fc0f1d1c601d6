"""Pins of the oracle's marching-cubes triangles (oracle.mesh) against what the
topology and geometry of a closed surface fix: every single-cell
configuration uses exactly its crossing edges and bounds its polygons by face
segments; closed solids give watertight meshes (each edge in two triangles,
in opposite directions) with the Euler characteristic of their topology (2
for a ball, 0 for a torus, 4 for two balls) and a positive enclosed volume
close to the solid's; a few configurations against hand-derived triangles."""
import itertools

import numpy as np
import pytest

import oracle


def cell_edge_ends(e):
    """Corner coordinates of cell edge e (4 a + u + 2 v)."""
    a, u, v = e // 4, e & 1, (e >> 1) & 1
    others = [x for x in range(3) if x != a]
    c0, c1 = [0, 0, 0], [0, 0, 0]
    c1[a] = 1
    c0[others[0]] = c1[others[0]] = u
    c0[others[1]] = c1[others[1]] = v
    return c0, c1


def key_of_cell_edge(e):
    """Key of cell edge e in a 2x2x2 lattice."""
    c0, _ = cell_edge_ends(e)
    return 3 * (c0[0] + 2 * (c0[1] + 2 * c0[2])) + e // 4


@pytest.mark.parametrize("case", range(1, 255))
def test_every_single_cell_configuration(case):
    occ = np.zeros((2, 2, 2), np.uint8)
    for b in range(8):
        if (case >> b) & 1:
            occ[(b >> 2) & 1, (b >> 1) & 1, b & 1] = 1
    keys = oracle.edges(occ)
    tris = oracle.mesh(occ, keys)
    assert len(tris) >= 1
    # exactly the crossing edges are used, each at least once
    assert set(tris.reshape(-1).tolist()) == set(range(len(keys)))
    # edges of the triangles used once form the polygons' boundary: each such
    # edge joins two cell edges on a common face
    cnt = {}
    for t in tris:
        for x, y in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            u = (min(x, y), max(x, y))
            cnt[u] = cnt.get(u, 0) + 1
    cell_edge = {key_of_cell_edge(e): e for e in range(12)}
    for (x, y), c in cnt.items():
        assert c in (1, 2)
        if c == 1:
            ex, ey = cell_edge[int(keys[x])], cell_edge[int(keys[y])]
            (a0, a1), (b0, b1) = cell_edge_ends(ex), cell_edge_ends(ey)
            share = [d for d in range(3) if a0[d] == a1[d] == b0[d] == b1[d]]
            assert share, (case, ex, ey)


def test_hand_derived_configurations():
    # one occupied corner: one triangle x-edge, y-edge, z-edge of corner 0,
    # facing away from it
    occ = np.zeros((2, 2, 2), np.uint8)
    occ[0, 0, 0] = 1
    keys = oracle.edges(occ)
    assert keys.tolist() == [0, 1, 2]
    assert oracle.mesh(occ, keys).tolist() == [[0, 1, 2]]
    # the bottom face occupied: the four vertical edges, one quad
    occ = np.zeros((2, 2, 2), np.uint8)
    occ[0] = 1
    keys = oracle.edges(occ)
    assert keys.tolist() == [2, 5, 8, 11]          # z-edges of corners 0..3
    tris = oracle.mesh(occ, keys)
    assert len(tris) == 2
    # the quad's normal is +z (away from the occupied layer)
    P = np.array([[c[0] + 0.0, c[1] + 0.0, 0.5] for c in ((0, 0), (1, 0), (0, 1), (1, 1))])
    for t in tris:
        n = np.cross(P[t[1]] - P[t[0]], P[t[2]] - P[t[0]])
        assert n[2] > 0 and abs(n[0]) + abs(n[1]) == 0
    # two corners on a face diagonal: two separate triangles
    occ = np.zeros((2, 2, 2), np.uint8)
    occ[0, 0, 0] = occ[0, 1, 1] = 1
    keys = oracle.edges(occ)
    tris = oracle.mesh(occ, keys)
    assert len(tris) == 2 and len(set(tris.reshape(-1).tolist())) == 6


def mesh_stats(occ):
    keys = oracle.edges(occ)
    tris = oracle.mesh(occ, keys)
    # vertex positions: edge midpoints
    nz, ny, nx = occ.shape
    lin, ax = keys // 3, keys % 3
    P = np.stack([lin % nx, (lin // nx) % ny, lin // (nx * ny)], 1).astype(np.float64)
    P[np.arange(len(keys)), ax] += 0.5
    directed = {}
    for t in tris:
        for x, y in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            directed[(int(x), int(y))] = directed.get((int(x), int(y)), 0) + 1
    V, F = len(keys), len(tris)
    E = len({(min(x, y), max(x, y)) for (x, y) in directed})
    vol = sum(np.dot(P[t[0]], np.cross(P[t[1]], P[t[2]])) for t in tris) / 6.0
    return keys, tris, directed, V - E + F, vol


def ball(n, centre, r):
    z, y, x = np.mgrid[:n, :n, :n]
    return ((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2 <= r * r)


@pytest.mark.parametrize("shape", ["ball", "torus", "two_balls", "random_blob"])
def test_closed_surfaces(shape):
    n = 24
    if shape == "ball":
        occ, chi = ball(n, (11.3, 12.1, 11.7), 7.6), 2
    elif shape == "torus":
        z, y, x = np.mgrid[:n, :n, :n]
        q = np.sqrt((x - 11.5) ** 2 + (y - 11.5) ** 2) - 6.5
        occ, chi = (q ** 2 + (z - 11.5) ** 2 <= 2.6 ** 2), 0
    elif shape == "two_balls":
        occ, chi = ball(n, (6.5, 7, 12), 4.3) | ball(n, (17, 16.5, 12), 4.6), 4
    else:
        rng = np.random.default_rng(7)
        occ = np.zeros((n, n, n), bool)
        for _ in range(6):
            occ |= ball(n, rng.uniform(8, 16, 3), rng.uniform(3, 5))
        chi = None
    occ = occ.astype(np.uint8)
    assert occ[0].max() == occ[-1].max() == occ[:, 0].max() == occ[:, :, -1].max() == 0
    keys, tris, directed, euler, vol = mesh_stats(occ)
    # watertight and consistently oriented: every edge once in each direction
    for (x, y), c in directed.items():
        assert c == 1 and directed.get((y, x)) == 1, (x, y)
    assert set(tris.reshape(-1).tolist()) == set(range(len(keys)))
    if chi is not None:
        assert euler == chi
    # outward orientation: the enclosed volume is positive and close to the
    # solid's (midpoint vertices: within a cell layer over the surface)
    assert vol > 0
    assert abs(vol - occ.sum()) < 0.6 * len(keys) ** 0.5 * 6 + 0.15 * occ.sum()


def test_counts_add_up_over_a_random_grid():
    """On a random (open) grid every crossing edge inside the lattice is used,
    and interior edges of the surface pair up with opposite directions."""
    rng = np.random.default_rng(3)
    occ = (rng.uniform(size=(9, 8, 7)) < 0.45).astype(np.uint8)
    keys, tris, directed, _, _ = mesh_stats(occ)
    assert set(tris.reshape(-1).tolist()) == set(range(len(keys)))
    for (x, y), c in directed.items():
        assert c == 1
