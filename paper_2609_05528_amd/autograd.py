"""A behind torch.autograd: forward is op_apply, backward is the hand-written A^T.

Because A is linear, the backward of A is A^T and the backward of A^T is A,
so derivatives of any order flow through the two HIP kernels.  Objectives
such as the ridge loss 1/2||A x - y||^2 + lambda/2 ||x||^2 (Sec. 9) can thus be
differentiated with respect to the emissivity coefficients.
"""
from __future__ import annotations

import torch

from . import op_apply, op_apply_adjoint


class RetardedTimeOp(torch.autograd.Function):
    """y = A x for x of shape [..., n_cols] (float32 CUDA)."""

    @staticmethod
    def forward(ctx, x, geom, order_mask=0):
        ctx.geom = geom
        ctx.order_mask = order_mask
        return op_apply(geom, x.contiguous(), order_mask=order_mask)

    @staticmethod
    def backward(ctx, gy):
        return RetardedTimeAdjointOp.apply(gy.contiguous(), ctx.geom, ctx.order_mask), None, None


class RetardedTimeAdjointOp(torch.autograd.Function):
    """x = A^T y for y of shape [..., n_rows]."""

    @staticmethod
    def forward(ctx, y, geom, order_mask=0):
        ctx.geom = geom
        ctx.order_mask = order_mask
        return op_apply_adjoint(geom, y.contiguous(), order_mask=order_mask)

    @staticmethod
    def backward(ctx, gx):
        return RetardedTimeOp.apply(gx.contiguous(), ctx.geom, ctx.order_mask), None, None


def retarded_time_apply(x, geom, order_mask=0):
    return RetardedTimeOp.apply(x, geom, order_mask)


def ridge_loss(x, y, geom, lam, order_mask=0):
    """1/2 ||A x - y||^2 + lam/2 ||x||^2 summed over the batch (differentiable)."""
    r = RetardedTimeOp.apply(x, geom, order_mask) - y
    return 0.5 * (r * r).sum() + 0.5 * lam * (x * x).sum()
