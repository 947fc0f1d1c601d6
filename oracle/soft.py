"""CPU oracle of the differentiable soft visual hull (TEST INFRASTRUCTURE).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the product path never imports it.  Plain PyTorch CPU ops in float64,
written as the definition reads, one camera at a time; the gradient is
torch.autograd through that definition (a library step), pinned in
tests/test_oracle_soft.py against central finite differences, closed forms
and the rotation's Rodrigues form.

The soft hull is the build's differentiable relative of the binary hull of
Sec. II-B-1 (not in the paper):
  * camera c maps a world point X to X_c = R_c X + t_c with
    R_c = exp([omega_c]x) R0_c and t_c = t0_c + tau_c (a 6-DoF perturbation of
    the calibrated pose), and to the continuous pixel position
    u = fx X_c.x / X_c.z + cx, v = fy X_c.y / X_c.z + cy, where pixel (x, y)
    covers [x, x+1) x [y, y+1) and so has its centre at (x + 0.5, y + 0.5);
  * p_c(X) = bilinear interpolation of sigmoid(L_c) between pixel centres at
    (u, v), pixels outside the image counting as 0, and p_c = 0 behind the
    camera;
  * o(X) = prod_c p_c(X) at each lattice sample, and the loss is
    sum_v (o_v - target_v)^2.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np
import torch

DT = torch.float64


def skew(w: torch.Tensor) -> torch.Tensor:
    """[w]x, the matrix with [w]x a = w x a."""
    z = torch.zeros((), dtype=w.dtype)
    return torch.stack([torch.stack([z, -w[2], w[1]]),
                        torch.stack([w[2], z, -w[0]]),
                        torch.stack([-w[1], w[0], z])])


def rotation(omega: torch.Tensor, R0: torch.Tensor) -> torch.Tensor:
    """exp([omega]x) R0 (matrix exponential, a library routine)."""
    return torch.linalg.matrix_exp(skew(omega)) @ R0


def lattice_points(origin: Sequence[float], h: float, lo: Sequence[int],
                   dims: Sequence[int]) -> torch.Tensor:
    """World positions [nz*ny*nx][3] of the lattice samples, x fastest:
    origin + (lo + index) * h per axis, in float64."""
    ax = [torch.as_tensor(float(origin[a]), dtype=DT) +
          (lo[a] + torch.arange(dims[a], dtype=DT)) * float(h) for a in range(3)]
    Z, Y, X = torch.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return torch.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], 1)


def bilinear(img: torch.Tensor, u: torch.Tensor, v: torch.Tensor) -> torch.Tensor:
    """Bilinear interpolation of img [H][W] between pixel centres at continuous
    pixel positions (u, v); taps outside the image are 0."""
    H, W = img.shape
    s, t = u - 0.5, v - 0.5
    x0, y0 = torch.floor(s), torch.floor(t)
    ax, ay = s - x0, t - y0
    x0, y0 = x0.long(), y0.long()
    out = torch.zeros_like(u)
    for dx, dy, wgt in ((0, 0, (1 - ax) * (1 - ay)), (1, 0, ax * (1 - ay)),
                        (0, 1, (1 - ax) * ay), (1, 1, ax * ay)):
        x, y = x0 + dx, y0 + dy
        inside = (x >= 0) & (x < W) & (y >= 0) & (y < H)
        val = img[y.clamp(0, H - 1), x.clamp(0, W - 1)]
        out = out + torch.where(inside, wgt * val, torch.zeros_like(u))
    return out


def camera_prob(logits_c: torch.Tensor, K_c: torch.Tensor, R_c: torch.Tensor, t_c: torch.Tensor,
                X: torch.Tensor) -> torch.Tensor:
    """p_c at the points X [V][3] for one camera (K_c = fx, fy, cx, cy)."""
    Xc = X @ R_c.T + t_c
    z = Xc[:, 2]
    front = z > 0
    zs = torch.where(front, z, torch.ones_like(z))
    u = K_c[0] * Xc[:, 0] / zs + K_c[2]
    v = K_c[1] * Xc[:, 1] / zs + K_c[3]
    p = bilinear(torch.sigmoid(logits_c), u, v)
    return torch.where(front, p, torch.zeros_like(p))


def occupancy(logits: torch.Tensor, K: torch.Tensor, R0: torch.Tensor, t0: torch.Tensor,
              omega: torch.Tensor, tau: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """o = prod over cameras of p_c at the points X."""
    o = torch.ones(X.shape[0], dtype=DT)
    for c in range(logits.shape[0]):
        o = o * camera_prob(logits[c], K[c], rotation(omega[c], R0[c]), t0[c] + tau[c], X)
    return o


def _tensors(logits, K, R0, t0, omega, tau):
    as64 = lambda a: torch.as_tensor(np.asarray(a, np.float64))
    return as64(logits), as64(K), as64(R0), as64(t0), as64(omega), as64(tau)


def soft_forward(logits, K, R0, t0, omega, tau, origin, h, lo, dims, target=None):
    """(o [V] float64 numpy, loss or None): the soft occupancy of the lattice
    and, with a target [V], sum (o - target)^2."""
    L, K, R0, t0, w, ta = _tensors(logits, K, R0, t0, omega, tau)
    X = lattice_points(origin, h, lo, dims)
    with torch.no_grad():
        o = occupancy(L, K, R0, t0, w, ta, X)
        loss = None
        if target is not None:
            tg = torch.as_tensor(np.asarray(target, np.float64).reshape(-1))
            loss = float(((o - tg) ** 2).sum())
    return o.numpy(), loss


def soft_grad(logits, K, R0, t0, omega, tau, origin, h, lo, dims, target=None,
              grad_occ=None) -> Tuple[float, np.ndarray, np.ndarray, np.ndarray]:
    """Gradient of sum (o - target)^2 (target given) or of sum grad_occ * o
    (a vector-Jacobian product) with respect to the logits [N][H][W], omega
    [N][3] and tau [N][3]; returns (objective, d_logits, d_omega, d_tau)."""
    L, K, R0, t0, w, ta = _tensors(logits, K, R0, t0, omega, tau)
    L.requires_grad_(True)
    w.requires_grad_(True)
    ta.requires_grad_(True)
    X = lattice_points(origin, h, lo, dims)
    o = occupancy(L, K, R0, t0, w, ta, X)
    if target is not None:
        tg = torch.as_tensor(np.asarray(target, np.float64).reshape(-1))
        obj = ((o - tg) ** 2).sum()
    else:
        obj = (torch.as_tensor(np.asarray(grad_occ, np.float64).reshape(-1)) * o).sum()
    gL, gw, gt = torch.autograd.grad(obj, (L, w, ta))
    return float(obj.detach()), gL.numpy(), gw.numpy(), gt.numpy()
