"""torch.autograd binding of the SDF pose / point adjoint.

``sdf_pose_loss(map, xi, pts)`` returns, per pose b, sum_j D(Exp(w_b) p_bj + t_b)^2 for
xi_b = (t_b, w_b); its backward uses the hand-written adjoint kernel (the point
gradients are recomputed in backward only when the points require them).
"""
from __future__ import annotations

import torch

from .mapcore import MAP_OK, MapError, map_last_error, map_sdf_pose_adjoint


def _run(m, xi, pts, with_points):
    B = xi.shape[0]
    loss = torch.empty(B, dtype=torch.float32, device=xi.device)
    gxi = torch.empty(B, 6, dtype=torch.float32, device=xi.device)
    gpts = torch.empty_like(pts) if with_points else None
    st = map_sdf_pose_adjoint(m.h, xi, pts, loss, gxi, gpts)
    if st != MAP_OK:
        raise MapError(st, map_last_error(m.h))
    return loss, gxi, gpts


class SdfPoseLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xi, pts, m):
        xi_c = xi.detach().contiguous()
        pts_c = pts.detach().contiguous()
        loss, gxi, _ = _run(m, xi_c, pts_c, with_points=False)
        ctx.m = m
        ctx.save_for_backward(xi_c, pts_c, gxi)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        xi, pts, gxi = ctx.saved_tensors
        g_xi = g_pts = None
        if ctx.needs_input_grad[1]:
            _, gxi, gpts = _run(ctx.m, xi, pts, with_points=True)
            g_pts = grad_loss[:, None, None] * gpts
        if ctx.needs_input_grad[0]:
            g_xi = grad_loss[:, None] * gxi
        return g_xi, g_pts, None


def sdf_pose_loss(m, xi, pts):
    """Per-pose squared-SDF loss of posed scans against map ``m`` (differentiable)."""
    return SdfPoseLoss.apply(xi, pts, m)
