"""Pins of the oracle's labelling (paper Sec. II-B-2: 26-adjacency components,
the minimum bounding box of each, the size filter of Eq. (1)).

The oracle's sequential union-find is checked against (a) its own BFS flood
fill, exhaustively on every 2x2x3 and 4x4x1 pattern, and (b) scipy's
``ndimage.label`` with a full 3x3x3 structuring element (the library routine
for 26-connectivity) on random and adversarial grids.  The filter, canonical
order (ascending smallest linear index) and boxes are checked by brute force.

Reading of Eq. (1): the equation and the sentence after it disagree; the
sentence (remove a set with fewer than T_np or more than T_nb voxels) is
followed, i.e. keep iff T_np <= N(S) <= T_nb.
"""
import itertools

import numpy as np
import pytest
from scipy import ndimage

import oracle

S26 = np.ones((3, 3, 3), bool)
UMAX = 0xFFFFFFFF


def canonical_partition(comp):
    """Relabel a component map so ids ascend with each component's first voxel."""
    flat = comp.reshape(-1)
    out = np.zeros_like(flat)
    mapping = {}
    for v in np.flatnonzero(flat):
        c = flat[v]
        if c not in mapping:
            mapping[c] = len(mapping) + 1
        out[v] = mapping[c]
    return out.reshape(comp.shape), len(mapping)


def brute_filter(occ, t_np, t_nb):
    lab, n = ndimage.label(occ, structure=S26)
    lab, n = canonical_partition(lab)
    rows, out_lab = [], np.zeros_like(lab)
    for c in range(1, n + 1):
        idx = np.argwhere(lab == c)                      # (k, j, i)
        cnt = idx.shape[0]
        if not (t_np <= cnt <= t_nb):
            continue
        K = len(rows) + 1
        out_lab[lab == c] = K
        lo = idx.min(0)[::-1]
        hi = idx.max(0)[::-1]
        first = int(np.flatnonzero((lab == c).reshape(-1))[0])
        rows.append([*lo, *hi, cnt, first])
    return out_lab, np.array(rows, np.int32).reshape(-1, 8)


def check_label(occ, t_np=1, t_nb=UMAX):
    occ_f, labels, rois, K = oracle.label(occ, t_np, t_nb)
    ref_lab, ref_rois = brute_filter(occ, t_np, t_nb)
    assert K == ref_rois.shape[0]
    np.testing.assert_array_equal(labels, ref_lab)
    np.testing.assert_array_equal(rois, ref_rois)
    np.testing.assert_array_equal(occ_f, (ref_lab > 0).astype(np.uint8))


@pytest.mark.parametrize("shape", [(3, 2, 2), (1, 4, 4)])
def test_exhaustive_small_patterns_against_bfs(shape):
    n = int(np.prod(shape))
    for bits in range(1 << n):
        occ = np.array([(bits >> b) & 1 for b in range(n)], np.uint8).reshape(shape)
        _, labels, _, K = oracle.label(occ, 1, UMAX)
        comp, nb = oracle.label_bfs(occ)
        assert K == nb
        np.testing.assert_array_equal(labels, comp)


def test_exhaustive_2x2x3_against_scipy():
    for bits in range(1 << 12):
        occ = np.array([(bits >> b) & 1 for b in range(12)], np.uint8).reshape(3, 2, 2)
        _, labels, _, K = oracle.label(occ, 1, UMAX)
        ref, n = canonical_partition(ndimage.label(occ, structure=S26)[0])
        assert K == n
        np.testing.assert_array_equal(labels, ref)


@pytest.mark.parametrize("seed", range(12))
def test_random_grids(seed):
    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in rng.integers(3, 17, size=3))
    dens = [0.05, 0.15, 0.3, 0.5, 0.7][seed % 5]
    occ = (rng.uniform(size=shape) < dens).astype(np.uint8)
    check_label(occ)
    check_label(occ, t_np=3, t_nb=40)


def test_diagonal_chain_is_one_component():
    occ = np.zeros((8, 8, 8), np.uint8)
    for t in range(8):
        occ[t, t, t] = 1                                   # vertex-sharing only
    _, labels, rois, K = oracle.label(occ, 1, UMAX)
    assert K == 1 and rois[0, 6] == 8
    assert ndimage.label(occ, structure=ndimage.generate_binary_structure(3, 2))[1] == 8  # 18-adj splits it


def test_checkerboard_is_one_component():
    k, j, i = np.indices((6, 7, 9))
    occ = ((i + j + k) % 2 == 0).astype(np.uint8)
    _, _, rois, K = oracle.label(occ, 1, UMAX)
    assert K == 1 and rois[0, 6] == occ.sum()
    check_label(occ)


def test_no_wraparound_at_borders():
    occ = np.zeros((4, 4, 5), np.uint8)
    occ[1, 1, 0] = 1
    occ[1, 1, 4] = 1                                       # same row, opposite ends
    occ[0, 0, 0] = 0
    _, _, _, K = oracle.label(occ, 1, UMAX)
    assert K == 2


def test_filter_bounds_are_inclusive():
    occ = np.zeros((10, 10, 30), np.uint8)
    occ[1, 1, 0:3] = 1        # 3 voxels
    occ[5, 5, 0:4] = 1        # 4 voxels
    occ[8, 8, 10:15] = 1      # 5 voxels
    occ[1, 8, 20:26] = 1      # 6 voxels
    for t_np, t_nb, expect in [(4, 5, [4, 5]), (3, 6, [3, 4, 5, 6]), (5, 5, [5]), (7, UMAX, []),
                               (1, 3, [3])]:
        occ_f, labels, rois, K = oracle.label(occ, t_np, t_nb)
        assert sorted(rois[:, 6].tolist()) == expect
        assert occ_f.sum() == sum(expect)
    check_label(occ, 4, 5)


def test_label_order_is_ascending_min_index():
    occ = np.zeros((6, 6, 6), np.uint8)
    occ[5, 0, 0] = occ[5, 0, 1] = 1      # late in raster order but...
    occ[0, 5, 5] = occ[1, 5, 5] = 1      # ...this one starts earlier
    occ[0, 0, 0] = occ[0, 0, 1] = 1
    _, labels, rois, K = oracle.label(occ, 1, UMAX)
    assert K == 3
    assert list(rois[:, 7]) == sorted(rois[:, 7])
    assert labels[0, 0, 0] == 1 and labels[0, 5, 5] == 2 and labels[5, 0, 0] == 3


def test_scene_coarse_grid(scene_cache):
    sc = scene_cache(2, 0)
    lat = oracle.Lattice(origin=sc.origin, h=sc.hc, lo=(0, 0, 0), dims=sc.coarse_dims)
    occ, _ = oracle.carve(sc.P32, oracle.pack(sc.masks), sc.W, sc.H, lat)
    check_label(occ, sc.t_np, sc.t_nb)
