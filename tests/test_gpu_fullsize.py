"""GPU results at the benchmark workloads' full sizes, in the launch configuration the
benchmark times, checked on sampled sources against the oracle.  Each sampled source is
evaluated by the oracle on its neighbourhood (itself plus every source whose box meets
one of its boxes), which leaves its terms unchanged (test_oracle_pins)."""
import sys

import numpy as np
import pytest

from conftest import neighbourhood

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


@pytest.fixture(scope="module")
def N():
    from oracle import newton
    return newton


def smallest(f, candidates, k):
    ptr = np.asarray(f.patch_ptr)
    px = [int(np.sum(f.boxes[ptr[s]:ptr[s + 1], 3].astype(np.int64) * f.boxes[ptr[s]:ptr[s + 1], 4]))
          for s in candidates]
    return [candidates[i] for i in np.argsort(px, kind="stable")[:k]]


def test_newton_field_1024src_full_size_sampled(B, N, synth):
    """One trust-region Newton step of all 1024 sources (others at their entry values), as
    the Newton benchmark runs it; sampled sources against the oracle's step."""
    f = synth.field_1024src()
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    say("case newton field_1024src full", plan.info())
    elbo, radius = plan.newton(theta, np.arange(f.n_src, dtype=np.int32), 1)
    th, elbo, radius = theta.cpu().numpy(), elbo.cpu().numpy(), radius.cpu().numpy()
    for s in smallest(f, list(range(0, f.n_src, 97)), 2):
        g, j = neighbourhood(f, s)
        say("  oracle newton source", s, "neighbourhood", g.n_src)
        row, fend, R = N.newton_steps(g, g.theta, j, 1)
        assert np.all(np.abs(th[s, :27] - row) <= 1e-6 * (1 + np.abs(row))), s
        np.testing.assert_allclose(elbo[s], fend, rtol=1e-9)
        assert radius[s] == R


def test_sweep_sky_region_20000src_full_size_sampled(B, O, synth):
    """One block-coordinate-ascent sweep over the 160-image region (conflict-free batches,
    two Newton steps per batch visit): monotone total ELBO, and the per-source ELBO of the
    final parameters on sampled sources against the oracle."""
    f = synth.sky_region_20000src()
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    ptr, src = plan.color_batches(seed=4)
    say("case sweep sky_region_20000src full", plan.info(), "batches", len(ptr) - 1)
    trace = plan.sweep(theta, ptr, src, 1, B.tr_params(newton_steps=2)).cpu().numpy()
    assert trace[1] >= trace[0]
    e = plan.elbo(theta).cpu().numpy()
    th = theta.cpu().numpy()
    assert np.any(th[:, :27] != f.theta[:, :27])
    hoods = [(s,) + neighbourhood(f, s, th) for s in range(0, f.n_src, 2999)]
    hoods.sort(key=lambda h: -h[1].n_src)            # the most crowded sampled sources
    for s, g, j in hoods[:3]:
        say("  oracle value source", s, "neighbourhood", g.n_src)
        v = O.source_value(O.Problem(g), j)
        np.testing.assert_allclose(e[s], v[0] + v[1], rtol=1e-9, atol=1e-12 * (abs(v[2]) + abs(v[1])))


def test_realistic_field_full_size_sampled(B, O, synth):
    """The 2000-source field with astrometry, sky maps and brightness-sized patches, at the
    benchmark's launch (graph replay): sampled ELBO and gradients against the oracle."""
    f = synth.sdss_field(2000, realistic=True)
    plan = B.Plan(f)
    plan.use_graph(True)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    say("case realistic field", plan.info())
    e, g = plan.elbo_grad(theta)
    e, g = e.cpu().numpy(), g.cpu().numpy()
    for s in (3, 1001, 1998):
        sub, j = neighbourhood(f, s)
        val, gref, gabs = O.source_grad(O.Problem(sub), j)
        np.testing.assert_allclose(e[s], val[0] + val[1], rtol=1e-9, atol=1e-12 * (abs(val[2]) + abs(val[1])))
        assert np.all(np.abs(g[s, :27] - gref) <= 1e-9 * np.abs(gref) + 1e-12 * gabs), s
