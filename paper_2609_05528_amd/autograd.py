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


class _RidgeNormalSolve(torch.autograd.Function):
    """x = (A^T A + lam I)^{-1} b on coefficient blocks; the matrix is symmetric, so the backward is
    the same solve (and derivatives of any order follow)."""

    @staticmethod
    def forward(ctx, b, geom, lam, tol, maxit):
        from .svd import ridge_solve
        ctx.args = (geom, lam, tol, maxit)
        x, _ = ridge_solve(geom, b.contiguous(), lam, tol=tol, maxit=maxit, normal_rhs=True)
        return x

    @staticmethod
    def backward(ctx, gx):
        geom, lam, tol, maxit = ctx.args
        return _RidgeNormalSolve.apply(gx.contiguous(), geom, lam, tol, maxit), None, None, None, None


class _TsvdProject(torch.autograd.Function):
    """x = V_t diag(sigma_t^-2) V_t^T b; symmetric, so the backward is the same map."""

    @staticmethod
    def forward(ctx, b, geom, svd, t, sigma_min):
        from .svd import tsvd_project
        ctx.args = (geom, svd, t, sigma_min)
        return tsvd_project(geom, svd, b.contiguous(), t=t, sigma_min=sigma_min)

    @staticmethod
    def backward(ctx, gx):
        geom, svd, t, sigma_min = ctx.args
        return _TsvdProject.apply(gx.contiguous(), geom, svd, t, sigma_min), None, None, None, None


def ridge_estimate(y, geom, lam, tol=1e-6, maxit=1000):
    """Ridge estimate x_hat = (A^T A + lam I)^{-1} A^T y (Sec. 9), differentiable in y: the backward
    is A applied to one more normal-equation solve."""
    return _RidgeNormalSolve.apply(RetardedTimeAdjointOp.apply(y.contiguous(), geom, 0), geom, lam, tol, maxit)


def tsvd_estimate(y, geom, svd, t=0, sigma_min=0.0):
    """TSVD estimate x_hat = V_t diag(sigma_t^-2) V_t^T A^T y (Sec. 9), differentiable in y."""
    return _TsvdProject.apply(RetardedTimeAdjointOp.apply(y.contiguous(), geom, 0), geom, svd, t, sigma_min)


class MixOp(torch.autograd.Function):
    """d = (L kron I) y for an order mixer of eq. (4); the backward is the transpose (L^T kron I)."""

    @staticmethod
    def forward(ctx, y, mixer):
        from .mixer import mix_apply
        ctx.mixer = mixer
        return mix_apply(mixer, y.contiguous())

    @staticmethod
    def backward(ctx, gd):
        return MixAdjointOp.apply(gd.contiguous(), ctx.mixer), None


class MixAdjointOp(torch.autograd.Function):
    """y = (L^T kron I) d; the backward is the mixer itself."""

    @staticmethod
    def forward(ctx, d, mixer):
        from .mixer import mix_adjoint
        ctx.mixer = mixer
        return mix_adjoint(mixer, d.contiguous())

    @staticmethod
    def backward(ctx, gy):
        return MixOp.apply(gy.contiguous(), ctx.mixer), None


def mixed_apply(x, geom, mixer, order_mask=0):
    """The mixed-arm operator (L kron I) A x (eq. (4) after eq. (3)), differentiable in x."""
    return MixOp.apply(RetardedTimeOp.apply(x.contiguous(), geom, order_mask), mixer)
