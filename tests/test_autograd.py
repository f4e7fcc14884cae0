"""The autograd wrapper: plumbing checked on the CPU with a stand-in plan whose ELBO is a
known analytic function, and on the GPU against the library's own gradient and HVP."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


class StandInPlan:
    """ELBO_s = -sum_i a_i exp(theta_si) + b_i theta_si^2 (a known function of theta)."""

    def __init__(self, S, seed=0):
        g = torch.Generator().manual_seed(seed)
        self.a = torch.rand(32, generator=g, dtype=torch.float64)
        self.b = torch.rand(32, generator=g, dtype=torch.float64)
        self.calls = {"elbo_grad": 0, "hvp": 0}

    def elbo_grad(self, theta, mode=1):
        self.calls["elbo_grad"] += 1
        e = -(self.a * torch.exp(theta) + self.b * theta ** 2).sum(1)
        g = -(self.a * torch.exp(theta) + 2 * self.b * theta)
        return e, g

    def hvp(self, theta, v):
        self.calls["hvp"] += 1
        return -(self.a * torch.exp(theta) + 2 * self.b) * v


def test_forward_backward_and_double_backward_plumbing():
    from paper_1801_10277_amd import torch_fn
    plan = StandInPlan(4)
    theta = torch.randn(4, 32, dtype=torch.float64, requires_grad=True)
    w = torch.randn(4, dtype=torch.float64)
    v = torch.randn(4, 32, dtype=torch.float64)
    e = torch_fn.elbo(theta, plan)
    (g,) = torch.autograd.grad((w * e).sum(), theta, create_graph=True)
    (h,) = torch.autograd.grad((g * v).sum(), theta)
    ref = theta.detach().clone().requires_grad_(True)
    er = -(plan.a * torch.exp(ref) + plan.b * ref ** 2).sum(1)
    (gr,) = torch.autograd.grad((w * er).sum(), ref, create_graph=True)
    (hr,) = torch.autograd.grad((gr * v).sum(), ref)
    torch.testing.assert_close(e, er, rtol=1e-15, atol=0)
    torch.testing.assert_close(g, gr, rtol=1e-14, atol=1e-14)
    torch.testing.assert_close(h, hr, rtol=1e-14, atol=1e-14)
    assert plan.calls == {"elbo_grad": 1, "hvp": 1}


@pytest.mark.gpu
def test_gpu_autograd_matches_library(synth):
    from paper_1801_10277_amd import binding as B, torch_fn
    assert torch.cuda.is_available()
    f = synth.tiny(S=3, n_bands=2, size=17, side=11, seed=5)
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda", requires_grad=True)
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device="cuda")
    v = torch.zeros(3, 32, dtype=torch.float64, device="cuda")
    v[:, :27] = torch.randn(3, 27, dtype=torch.float64, device="cuda")
    e = torch_fn.elbo(theta, plan)
    (g,) = torch.autograd.grad((w * e).sum(), theta, create_graph=True)
    (h,) = torch.autograd.grad((g * v).sum(), theta)
    e0, g0 = plan.elbo_grad(theta.detach())
    hv = plan.hvp(theta.detach(), v)
    torch.testing.assert_close(e.detach(), e0, rtol=0, atol=0)
    torch.testing.assert_close(g.detach(), w[:, None] * g0, rtol=1e-15, atol=0)
    torch.testing.assert_close(h, w[:, None] * hv, rtol=1e-15, atol=0)
