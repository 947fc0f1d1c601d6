"""Differentiable soft visual hull as torch.autograd Functions over the C ABI
(``fvv_soft_forward`` / ``fvv_soft_backward``; the model is stated in
include/fvv.h).  Argument marshalling only: the forward and the adjoint run in
the library's HIP kernels.  Logits live on the device; the pose perturbations
omega and tau are small host-side parameter sets (the library forms the
rotations in double on the host), so a device omega/tau is copied to the host
at each call.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Grid, soft_cameras


class SoftHull:
    """A calibrated rig (K [N][4] = fx, fy, cx, cy; R0 [N][3][3]; t0 [N][3];
    image W x H) and a lattice, evaluated on one library context."""

    def __init__(self, ctx, grid: Grid, K, R0, t0, W: int, H: int):
        self.ctx, self.grid = ctx, grid
        self.K = np.asarray(K, np.float64)
        self.R0 = np.asarray(R0, np.float64)
        self.t0 = np.asarray(t0, np.float64)
        self.W, self.H = int(W), int(H)

    def cameras(self, omega, tau):
        host = lambda a: (a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else np.asarray(a))
        return soft_cameras(self.K, self.R0, self.t0, host(omega), host(tau))

    def occupancy(self, logits, omega, tau):
        """Soft occupancy o [nz*ny*nx] (x fastest), differentiable in logits,
        omega and tau."""
        return _SoftOcc.apply(self, logits, omega, tau)

    def l2_loss(self, logits, omega, tau, target):
        """sum (o - target)^2 as a 0-dim float64 tensor, differentiable in
        logits, omega and tau (the fused kernels: no occupancy is stored)."""
        return _SoftL2.apply(self, logits, omega, tau, target)


def _pose_grads(gp, omega, tau):
    """Gradients for omega and tau in their own dtype and device (None for a
    pose given as a plain array, which autograd does not track)."""
    like = lambda g, a: (g.to(device=a.device, dtype=a.dtype) if isinstance(a, torch.Tensor)
                         else None)
    return like(gp[:, :3].contiguous(), omega), like(gp[:, 3:].contiguous(), tau)


def _check_logits(hull, logits):
    if not (isinstance(logits, torch.Tensor) and logits.is_cuda and logits.dtype == torch.float32
            and logits.is_contiguous() and tuple(logits.shape) == (hull.K.shape[0], hull.H, hull.W)):
        raise ValueError("logits must be a contiguous float32 CUDA tensor [N][H][W]")


class _SoftOcc(torch.autograd.Function):
    @staticmethod
    def forward(ctx, hull: SoftHull, logits, omega, tau):
        _check_logits(hull, logits)
        cams = hull.cameras(omega, tau)
        occ = torch.empty(hull.grid.size, dtype=torch.float32, device=logits.device)
        hull.ctx.soft_forward(hull.grid, cams, hull.W, hull.H, logits, occ=occ)
        ctx.hull, ctx.cams = hull, cams
        ctx.save_for_backward(logits, omega if isinstance(omega, torch.Tensor) else None,
                              tau if isinstance(tau, torch.Tensor) else None)
        return occ

    @staticmethod
    def backward(ctx, grad_occ):
        logits, omega, tau = ctx.saved_tensors
        hull = ctx.hull
        gl = torch.empty_like(logits)
        gp = torch.empty((len(ctx.cams), 6), dtype=torch.float64, device=logits.device)
        hull.ctx.soft_backward(hull.grid, ctx.cams, hull.W, hull.H, logits, gl, gp,
                               grad_occ=grad_occ.detach().to(torch.float32).contiguous())
        gw, gt = _pose_grads(gp, omega, tau)
        return None, gl, gw, gt


class _SoftL2(torch.autograd.Function):
    @staticmethod
    def forward(ctx, hull: SoftHull, logits, omega, tau, target):
        _check_logits(hull, logits)
        cams = hull.cameras(omega, tau)
        target = target.detach().to(torch.float32).contiguous()
        loss = torch.empty(1, dtype=torch.float64, device=logits.device)
        hull.ctx.soft_forward(hull.grid, cams, hull.W, hull.H, logits, target=target, loss=loss)
        ctx.hull, ctx.cams = hull, cams
        ctx.save_for_backward(logits, target, omega if isinstance(omega, torch.Tensor) else None,
                              tau if isinstance(tau, torch.Tensor) else None)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        logits, target, omega, tau = ctx.saved_tensors
        hull = ctx.hull
        gl = torch.empty_like(logits)
        gp = torch.empty((len(ctx.cams), 6), dtype=torch.float64, device=logits.device)
        scale = g.detach().to(torch.float64).reshape(1).contiguous()
        hull.ctx.soft_backward(hull.grid, ctx.cams, hull.W, hull.H, logits, gl, gp, target=target,
                               scale=scale)
        gw, gt = _pose_grads(gp, omega, tau)
        return None, gl, gw, gt, None
