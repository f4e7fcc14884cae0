"""PyTorch autograd wrappers of the HIP ELBO path.

Two functions, with different derivative semantics:

* `total_elbo(theta, plan)` is the ELBO of the whole field (Eq. (1): every covered pixel
  once, minus every source's KL), a scalar.  Its gradient is exact: a pixel term depends on
  theta_s only if the pixel lies in one of s's boxes, and those pixel terms are exactly the
  ones ELBO_s sums, so d total / d theta_s = d ELBO_s / d theta_s, which the library's
  adjoint returns.  It is differentiable once (the Hessian of the total has blocks between
  overlapping sources, which the library does not form).

* `elbo(theta, plan)` returns the per-source ELBO_s (a [S] tensor), each differentiated in
  its own source's parameters only, as in block coordinate ascent (Section IV-D): the other
  sources are treated as constants of ELBO_s.  So the gradient of sum_s w_s ELBO_s with
  respect to theta_s is w_s d ELBO_s / d theta_s, and the cross terms d ELBO_t / d theta_s
  of overlapping sources t are left out on purpose.  Its backward is the adjoint's gradient
  (computed in the same call as the forward) and the backward of that backward is the
  tangent-adjoint Hessian-vector product of each source's own block, so
  `torch.autograd.grad(..., create_graph=True)` followed by another grad gives exact
  second derivatives of the per-source blocks.

PyTorch only carries the tensors and the stream; every number is computed by libceleste.
"""
import torch
from torch.autograd.function import once_differentiable

from . import binding as B


class _ELBO(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, plan, mode):
        elbo, grad = plan.elbo_grad(theta.detach().contiguous(), mode=mode)
        ctx.plan = plan
        ctx.save_for_backward(theta, grad)
        return elbo

    @staticmethod
    def backward(ctx, g_out):
        theta, grad = ctx.saved_tensors
        return _ScaledGrad.apply(theta, grad, g_out, ctx.plan), None, None


class _ScaledGrad(torch.autograd.Function):
    """g_out[s] * d ELBO_s / d theta_s, differentiable once more through the HVP."""

    @staticmethod
    def forward(ctx, theta, grad, g_out, plan):
        ctx.plan = plan
        ctx.save_for_backward(theta, grad, g_out)
        return g_out[:, None] * grad

    @staticmethod
    def backward(ctx, gg):
        theta, grad, g_out = ctx.saved_tensors
        d_theta = d_gout = None
        if ctx.needs_input_grad[0]:
            hv = ctx.plan.hvp(theta.detach().contiguous(), gg.detach().contiguous())
            d_theta = g_out[:, None] * hv
        if ctx.needs_input_grad[2]:
            d_gout = (gg * grad).sum(dim=1)
        return d_theta, None, d_gout, None


class _TotalELBO(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, plan):
        th = theta.detach().contiguous()
        total = plan.total_elbo(th)[0]
        _, grad = plan.elbo_grad(th)
        ctx.save_for_backward(grad)
        return total

    @staticmethod
    @once_differentiable
    def backward(ctx, g_out):
        (grad,) = ctx.saved_tensors
        return g_out * grad, None


def elbo(theta, plan, mode=B.CELESTE_BATCHED):
    """Per-source ELBO_s of theta ([S, 48] float64 on the plan's device), each differentiated
    in its own source's parameters only (the other sources held fixed)."""
    return _ELBO.apply(theta, plan, mode)


def total_elbo(theta, plan):
    """Total ELBO of the field (a 0-d tensor) with its exact gradient; differentiable once."""
    return _TotalELBO.apply(theta, plan)


def hvp(theta, v, plan):
    """Block-diagonal Hessian-vector product d^2 ELBO_s / d theta_s^2 v_s."""
    return plan.hvp(theta.detach().contiguous(), v.detach().contiguous())
