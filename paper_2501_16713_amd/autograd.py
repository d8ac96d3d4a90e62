"""torch.autograd wrappers of the warp and the nonrigid SENSE operator.

The backward passes call the library's hand-written adjoint kernels, so
gradients with respect to the image use the exact adjoint T^H / A^H (the
forward-adjoint pair of Eq. 7-9) and gradients with respect to the
displacement fields use the derivative of the interpolation weights
(PyTorch's convention for complex tensors: grad = dL/dRe + i dL/dIm).

    plan = Plan(shape, ncoils, nphases)
    y = warp(plan, x, d)                    # T_d x, differentiable in x and d
    y = sense(plan, x, ds, S, trajs)        # [A_0; ...; A_{P-1}] x, in x and ds
"""
from __future__ import annotations

import torch

from .ops import Plan


class WarpFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, d, plan: Plan):
        motion = plan.motion(d.detach())
        ctx.plan, ctx.motion = plan, motion
        ctx.save_for_backward(x)
        return plan.warp(x.detach(), motion)

    @staticmethod
    def backward(ctx, gy):
        (x,) = ctx.saved_tensors
        gy = gy.contiguous()
        gx = ctx.plan.warp_adjoint(gy, ctx.motion) if ctx.needs_input_grad[0] else None
        gd = ctx.plan.warp_grad_d(x.detach(), gy, ctx.motion) if ctx.needs_input_grad[1] else None
        return gx, gd, None


class SenseFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, ds, S, plan: Plan, trajs):
        motions = [plan.motion(ds[p].detach()) for p in range(ds.shape[0])]
        ctx.plan, ctx.motions, ctx.trajs = plan, motions, trajs
        ctx.save_for_backward(x, S)
        return plan.sense_forward(x.detach(), motions, S, trajs)

    @staticmethod
    def backward(ctx, gy):
        x, S = ctx.saved_tensors
        want_x, want_d = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gx, gd = ctx.plan.sense_grad(x.detach(), ctx.motions, S, ctx.trajs, gy.contiguous(),
                                     want_x=want_x, want_d=want_d)
        return gx, gd, None, None, None


def warp(plan: Plan, x: torch.Tensor, d: torch.Tensor) -> torch.Tensor:
    """T_d x with gradients for x (T^H) and d."""
    return WarpFunction.apply(x, d, plan)


def sense(plan: Plan, x: torch.Tensor, ds: torch.Tensor, S: torch.Tensor, trajs) -> torch.Tensor:
    """Stacked nonrigid SENSE model; ds is [P][ndim][*shape]; returns
    [sum_p M_p][C].  Gradients for x (A^H) and ds."""
    return SenseFunction.apply(x, ds, S, plan, list(trajs))
