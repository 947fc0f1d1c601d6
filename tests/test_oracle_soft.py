"""Pins of the soft-hull oracle (oracle/soft.py) against what the definition
and the mathematics fix: the rotation's Rodrigues form, bilinear values at
pixel centres, midpoints and borders, a constant-logit closed form, points
behind a camera, and the autograd gradient against central finite
differences in float64 (logits and all six pose components)."""
import math

import numpy as np
import pytest
import torch

import scenes
from oracle import soft

DT = torch.float64


def rodrigues(w):
    """exp([w]x) by its closed form I + sin(t)/t K + (1 - cos t)/t^2 K^2."""
    w = np.asarray(w, np.float64)
    t = np.linalg.norm(w)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if t < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + math.sin(t) / t * K + (1 - math.cos(t)) / t ** 2 * K @ K


@pytest.mark.parametrize("w", [(0, 0, 0), (1e-9, -2e-9, 3e-9), (0.01, -0.02, 0.005), (0.7, 0.2, -1.1),
                               (math.pi / 2, 0, 0)])
def test_rotation_is_rodrigues(w):
    R0 = torch.as_tensor(scenes.tiny_rig(4)[1].R)
    R = soft.rotation(torch.as_tensor(w, dtype=DT), R0).numpy()
    np.testing.assert_allclose(R, rodrigues(w) @ R0.numpy(), atol=1e-12)
    np.testing.assert_allclose(R.T @ R, np.eye(3), atol=1e-12)
    assert abs(np.linalg.det(R) - 1) < 1e-12


def test_bilinear_centres_midpoints_and_borders():
    rng = np.random.default_rng(3)
    img = torch.as_tensor(rng.uniform(size=(5, 7)))
    # at a pixel centre the value is that pixel's
    ys, xs = torch.meshgrid(torch.arange(5), torch.arange(7), indexing="ij")
    got = soft.bilinear(img, xs.reshape(-1).double() + 0.5, ys.reshape(-1).double() + 0.5)
    np.testing.assert_allclose(got.numpy(), img.reshape(-1).numpy(), atol=1e-15)
    # midway between four centres: their mean
    got = soft.bilinear(img, torch.tensor([2.0]), torch.tensor([3.0]))
    assert abs(float(got) - float(img[2:4, 1:3].mean())) < 1e-15
    # a quarter pixel outside the left border: 3/4 of the border pixel
    got = soft.bilinear(img, torch.tensor([0.25]), torch.tensor([2.5]))
    assert abs(float(got) - 0.75 * float(img[2, 0])) < 1e-15
    # beyond half a pixel outside: 0
    got = soft.bilinear(img, torch.tensor([-0.5, 7.5, 3.0, 3.0]), torch.tensor([2.5, 2.5, -0.5, 5.5]))
    assert float(got.abs().max()) == 0.0


def small_case(n_cams=4, dims=(6, 5, 4), seed=0):
    s = scenes.scene_soft(seed, n_cams=n_cams)
    K, R0, t0 = s.base_pose()
    # a small box of samples at the centre of the scene's lattice
    lo = tuple(s.lo[a] + (s.dims[a] - dims[a]) // 2 for a in range(3))
    return s, K, R0, t0, lo, dims


def test_constant_logits_closed_form():
    s, K, R0, t0, lo, dims = small_case()
    L = np.full_like(s.logits, 0.8)
    o, _ = soft.soft_forward(L, K, R0, t0, s.omega, s.tau, s.origin, s.h, lo, dims)
    # every sample projects well inside every image, so p_c = sigmoid(L) (L is float32 0.8)
    assert abs(o - (1 / (1 + math.exp(-float(np.float32(0.8))))) ** 4).max() < 1e-14


def test_points_behind_a_camera_are_empty():
    s, K, R0, t0, lo, dims = small_case()
    t0 = t0.copy()
    t0[2, 2] = -20.0          # camera 2 now has every sample behind it
    o, _ = soft.soft_forward(np.full_like(s.logits, 5.0), K, R0, t0, s.omega, s.tau, s.origin, s.h,
                             lo, dims)
    assert float(np.abs(o).max()) == 0.0


def test_zero_loss_at_its_own_occupancy():
    s, K, R0, t0, lo, dims = small_case()
    o, _ = soft.soft_forward(s.logits, K, R0, t0, s.omega, s.tau, s.origin, s.h, lo, dims)
    loss, gL, gw, gt = soft.soft_grad(s.logits, K, R0, t0, s.omega, s.tau, s.origin, s.h, lo, dims,
                                      target=o)
    assert loss < 1e-28 and np.abs(gL).max() < 1e-14 and np.abs(gw).max() < 1e-12


def test_gradient_matches_central_differences():
    s, K, R0, t0, lo, dims = small_case(dims=(8, 7, 6))
    target = (np.random.default_rng(1).uniform(size=int(np.prod(dims))) < 0.3).astype(np.float64)
    args = (K, R0, t0)
    loss, gL, gw, gt = soft.soft_grad(s.logits, *args, s.omega, s.tau, s.origin, s.h, lo, dims,
                                      target=target)

    def f(L, w, t):
        return soft.soft_forward(L, *args, w, t, s.origin, s.h, lo, dims, target)[1]

    eps = 1e-6
    w0, t0_ = s.omega.astype(np.float64), s.tau.astype(np.float64)
    L0 = s.logits.astype(np.float64)
    for c in range(4):
        for a in range(3):
            for (arr, g) in ((w0, gw), (t0_, gt)):
                hi, lo_ = arr.copy(), arr.copy()
                hi[c, a] += eps
                lo_[c, a] -= eps
                fd = (f(L0, hi, t0_) - f(L0, lo_, t0_)) / (2 * eps) if arr is w0 else \
                    (f(L0, w0, hi) - f(L0, w0, lo_)) / (2 * eps)
                assert abs(fd - g[c, a]) <= 1e-6 * max(1.0, abs(g[c, a])), (c, a, fd, g[c, a])
    # logits: the pixels with the largest gradients
    idx = np.argsort(-np.abs(gL).reshape(-1))[:12]
    for flat in idx:
        hi, lo_ = L0.copy().reshape(-1), L0.copy().reshape(-1)
        hi[flat] += eps
        lo_[flat] -= eps
        fd = (f(hi.reshape(L0.shape), w0, t0_) - f(lo_.reshape(L0.shape), w0, t0_)) / (2 * eps)
        g = gL.reshape(-1)[flat]
        assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (flat, fd, g)


def test_vector_jacobian_product_of_the_loss():
    s, K, R0, t0, lo, dims = small_case()
    target = np.zeros(int(np.prod(dims)))
    o, _ = soft.soft_forward(s.logits, K, R0, t0, s.omega, s.tau, s.origin, s.h, lo, dims)
    a = soft.soft_grad(s.logits, K, R0, t0, s.omega, s.tau, s.origin, s.h, lo, dims, target=target)
    b = soft.soft_grad(s.logits, K, R0, t0, s.omega, s.tau, s.origin, s.h, lo, dims,
                       grad_occ=2 * (o - target))
    for x, y in zip(a[1:], b[1:]):
        np.testing.assert_allclose(x, y, rtol=1e-12, atol=1e-15)
