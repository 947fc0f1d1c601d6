"""Pins of the oracle's pixel arithmetic, silhouette packing and lattice sizes.

The occupancy test (paper Sec. II-B) needs the pixel that a voxel projects to:
the exact floor of the real quotient a/w.  These tests pin the oracle's floor
against exact rational arithmetic, its bit packing against numpy's packbits,
and the corner-anchored lattice convention against the voxel counts the paper
prints (Sec. II-B-1 / II-B-3, golden fixture).
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")


def _exact_floor(a: np.float32, w: np.float32) -> int:
    return math.floor(Fraction(float(a)) / Fraction(float(w)))


def test_floor_div_random_against_fractions():
    rng = np.random.default_rng(1)
    a = rng.uniform(-5000, 5000, 4000).astype(np.float32)
    w = rng.uniform(0.05, 200, 4000).astype(np.float32)
    for ai, wi in zip(a, w):
        assert oracle.floor_div(ai, wi) == _exact_floor(ai, wi)


def test_floor_div_near_integers_against_fractions():
    """Quotients within a few ulp of an integer: the cases a naive floor of a
    rounded float quotient gets wrong."""
    rng = np.random.default_rng(2)
    bad_naive = 0
    for _ in range(3000):
        w = np.float32(rng.uniform(0.5, 60))
        n = int(rng.integers(-100, 4000))
        a0 = np.float32(np.float32(n) * w)
        for a in (np.nextafter(a0, np.float32(-np.inf)), a0, np.nextafter(a0, np.float32(np.inf))):
            exact = _exact_floor(a, w)
            assert oracle.floor_div(a, w) == exact
            bad_naive += int(math.floor(float(np.float32(a / w))) != exact)
    assert bad_naive > 0, "the adversarial set must contain cases that a float quotient floors wrongly"


def test_floor_div_exact_multiples():
    for w in (np.float32(3.0), np.float32(0.1), np.float32(7.25), np.float32(1e-3)):
        for n in range(-50, 2000, 7):
            a = np.float32(n) * w
            if Fraction(float(a)) == n * Fraction(float(w)):
                assert oracle.floor_div(a, w) == n


@pytest.mark.parametrize("W", [1, 31, 32, 33, 320, 1920, 3841])
def test_pack_against_packbits(W):
    rng = np.random.default_rng(W)
    masks = (rng.uniform(size=(3, 7, W)) < 0.4).astype(np.uint8)
    words = oracle.pack(masks)
    wpr = (W + 31) // 32
    padded = np.zeros((3, 7, wpr * 32), np.uint8)
    padded[..., :W] = masks
    ref = np.packbits(padded, axis=-1, bitorder="little").view("<u4")
    assert words.shape == (3, 7, wpr)
    np.testing.assert_array_equal(words, ref)


def test_lattice_size_matches_printed_counts():
    g = json.load(open(GOLDEN))
    sp = g["sparse_hull"]
    dims = [scenes.lattice_dims(e, sp["voxel_um"]) for e in sp["extent_m"]]
    assert dims == [360, 360, 180]
    n = int(np.prod(dims))
    assert n == 23_328_000
    assert round(n / 1e7, 1) == sp["voxels_tested_printed"] / 1e7
    # the paper gives the dense/sparse occupancy ratio as about 15: (50/20)^3 = 15.6
    dn = g["dense_hull"]
    assert abs((sp["voxel_um"] / dn["voxel_um"]) ** 3 - dn["occupied_ratio_printed"]) < 1.0
    assert abs(dn["voxels_occupied_printed"] / sp["voxels_occupied_printed"] - dn["occupied_ratio_printed"]) < 1.0


def test_table2_rows_sum_to_table1():
    t = json.load(open(GOLDEN))["timing_ms"]
    tot = np.sum(np.array(list(t["table2"].values())), axis=0)
    np.testing.assert_allclose(tot, t["table1_proposed"], atol=0.011)
