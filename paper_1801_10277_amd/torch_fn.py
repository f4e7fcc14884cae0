"""PyTorch autograd wrapper of the HIP ELBO path.

`elbo(theta, plan)` returns the per-source ELBO_s (a [S] tensor); its backward is the
hand-written adjoint's gradient (computed in the same call as the forward), and the
backward of that backward is the tangent-adjoint Hessian-vector product, so
`torch.autograd.grad(..., create_graph=True)` followed by another grad gives exact
second derivatives of the per-source blocks.  PyTorch only carries the tensors and the
stream; every number is computed by libceleste.
"""
import torch

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


def elbo(theta, plan, mode=B.CELESTE_BATCHED):
    """Per-source ELBO_s of theta ([S, 32] float64 on the plan's device)."""
    return _ELBO.apply(theta, plan, mode)


def hvp(theta, v, plan):
    """Block-diagonal Hessian-vector product d^2 ELBO_s / d theta_s^2 v_s."""
    return plan.hvp(theta.detach().contiguous(), v.detach().contiguous())
