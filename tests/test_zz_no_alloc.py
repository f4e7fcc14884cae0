"""celeste_elbo_grad_noalloc (the entry point that allocates nothing: partial sums in the
library's static device scratch) against celeste_elbo_grad, through the C ABI."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1801_10277_amd import binding
    assert torch.cuda.is_available()
    return binding


def test_noalloc_equals_elbo_grad_on_two_calls_larger_then_smaller(B, synth):
    """Two calls in a row on one device, the second on a smaller problem (fewer work items,
    so the static scratch still holds the first call's larger partial sums): both equal the
    plan-memory entry point bitwise, ELBO and gradient."""
    big = synth.tiny(S=6, n_bands=3, size=48, side=27, seed=301)
    small = synth.tiny(S=2, n_bands=2, size=17, side=9, seed=302)
    for name, f in (("larger", big), ("smaller", small)):
        plan = B.Plan(f)
        theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
        say("case noalloc", name, plan.info()["n_items"], "items")
        e0, g0 = plan.elbo_grad(theta)
        e1 = torch.full_like(e0, np.nan)
        g1 = torch.full_like(g0, np.nan)
        plan.elbo_grad_noalloc(theta, elbo=e1, grad=g1)
        torch.cuda.synchronize()
        assert torch.equal(e0, e1) and torch.equal(g0, g1), name


def test_noalloc_dynamic_queue_and_active_mask(B, synth):
    """With the counter-based work queue (its counter lives in the scratch too) and an
    active mask: equal to celeste_elbo_grad, inactive outputs untouched."""
    f = synth.tiny(S=5, n_bands=2, size=40, side=21, seed=303)
    plan = B.Plan(f)
    plan.set_launch(chunk=64, waves_per_block=2, grid_blocks=64, dynamic=1, strip_rows=8)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    act = torch.tensor([1, 0, 1, 1, 0], dtype=torch.uint8, device="cuda")
    say("case noalloc dynamic + active")
    for _ in range(2):
        e0 = torch.full((5,), 5.0, dtype=torch.float64, device="cuda")
        g0 = torch.full((5, 48), 2.0, dtype=torch.float64, device="cuda")
        e1, g1 = e0.clone(), g0.clone()
        plan.elbo_grad(theta, active=act, elbo=e0, grad=g0)
        plan.elbo_grad_noalloc(theta, active=act, elbo=e1, grad=g1)
        torch.cuda.synchronize()
        assert torch.equal(e0, e1) and torch.equal(g0, g1)
        assert torch.all(e1[[1, 4]] == 5.0) and torch.all(g1[[1, 4]] == 2.0)


def test_noalloc_rejects_problems_beyond_the_scratch(B, synth):
    """The 2000-source field at 4-row strips needs 129 735 work items (11 MiB of partial
    sums): CELESTE_ESCRATCH, nothing run, outputs untouched; at 16-row strips (38 560 items)
    it runs and equals celeste_elbo_grad."""
    f = synth.field_2000src()
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    plan.set_launch(strip_rows=4)
    say("case noalloc too large", plan.info()["n_items"], "items")
    e = torch.full((f.n_src,), 3.0, dtype=torch.float64, device="cuda")
    g = torch.full((f.n_src, 48), 4.0, dtype=torch.float64, device="cuda")
    with pytest.raises(B.CelesteError) as err:
        plan.elbo_grad_noalloc(theta, elbo=e, grad=g)
    assert err.value.code == B.CELESTE_ESCRATCH
    torch.cuda.synchronize()
    assert torch.all(e == 3.0) and torch.all(g == 4.0)
    plan.set_launch(strip_rows=16)
    say("case noalloc field_2000src", plan.info()["n_items"], "items")
    e0, g0 = plan.elbo_grad(theta)
    plan.elbo_grad_noalloc(theta, elbo=e, grad=g)
    torch.cuda.synchronize()
    assert torch.equal(e0, e) and torch.equal(g0, g)
