"""torch.autograd.Function around the VGICP cost (Eq. (2)) and its hand-written backward kernel.

VGICPCost.apply(xi_source, xi_target, xyz, cov, vmap, T_target, T_source, binary, precision)
returns the cost e of one factor evaluated at T_source Exp(xi_source) and (binary)
T_target Exp(xi_target). Its gradients are
  d e / d xi_source, d e / d xi_target   (se(3) tangents, [omega; rho], float64 (6,))
  d e / d xyz                            (per source point, float32 (3, n))
with the correspondences held at those found by the forward pass. The library does all of the
arithmetic (the retraction, the backward kernel and the map of the gradient to the tangent
coordinates through the SE(3) right Jacobian); this module only moves tensors.
"""
from __future__ import annotations

import torch

from . import vgicp as V


class VGICPCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xi_source, xi_target, xyz, cov, vmap, T_target, T_source, binary,
                precision=V.VGICP_ACC_FP64):
        xs = xi_source.detach().to("cpu", torch.float64).numpy()
        xt = xi_target.detach().to("cpu", torch.float64).numpy() if binary else None
        Ts = V.vgicp_se3_retract(T_source, xs)
        Tt = V.vgicp_se3_retract(T_target, xt) if binary else T_target
        r = V.vgicp_evaluate(vmap, xyz, cov, Tt, Ts, precision, want_corr=True)
        ctx.save_for_backward(xyz, cov, r["corr"])
        ctx.vmap = vmap
        ctx.poses = (T_target, T_source)
        ctx.binary = bool(binary)
        ctx.xi = (xs, xt)
        ctx.precision = V.VGICP_MATH_FP64 if precision == V.VGICP_MATH_FP64 else V.VGICP_ACC_FP64
        ctx.xi_device = xi_source.device
        return r["err"].reshape(())

    @staticmethod
    def backward(ctx, grad):
        xyz, cov, corr = ctx.saved_tensors
        g = grad.detach().reshape(1).to(device=xyz.device, dtype=torch.float64).contiguous()
        Tt, Ts = ctx.poses
        xs, xt = ctx.xi
        gxi, gp = V.vgicp_backward_tangent(ctx.vmap, xyz, cov, Tt, Ts, xt, xs, ctx.binary, corr,
                                           g, ctx.precision,
                                           want_points=ctx.needs_input_grad[2])
        g_s = gxi[:6].to(ctx.xi_device)
        g_t = gxi[6:].to(ctx.xi_device) if ctx.binary else None
        return g_s, g_t, gp, None, None, None, None, None, None


def vgicp_cost(xi_source, xi_target, xyz, cov, vmap, T_target, T_source, binary,
               precision=V.VGICP_ACC_FP64):
    return VGICPCost.apply(xi_source, xi_target, xyz, cov, vmap, T_target, T_source, binary,
                           precision)
