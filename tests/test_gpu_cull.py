"""GPU: the strip kernels' component culling against the FP64 oracle.

The strip kernels leave out of a work item every Gaussian whose quadratic form exceeds 100
on all of the item's pixels (below exp(-50) of its own peak there); the oracle evaluates
every Gaussian on every pixel.  On a field of wide boxes around compact sources many
(item, Gaussian) pairs are culled, and an odd number of live galaxy components in a PSF
group is padded with the zero component, so both code paths run.  Tolerance as in the
other parity tests: |gpu - oracle| <= 1e-9 |oracle| + 1e-12 G, G the oracle's sum of
|per-visit terms|.
"""
import sys

import numpy as np
import pytest

from conftest import hessian_within

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

REL = 1e-9
FLOOR = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    from paper_1801_10277_amd import binding
    assert torch.cuda.is_available()
    return binding


def within(got, ref, absum, what):
    err = np.abs(got - ref)
    bound = REL * np.abs(ref) + FLOOR * absum
    bad = err > bound
    assert not bad.any(), "%s: max err/bound %.3g at %s" % (
        what, (err / np.maximum(bound, 1e-300)).max(), np.argwhere(bad)[:5].tolist())


def wide_boxes(synth):
    # three sources in a 72 x 72 region with 61-pixel boxes: 4 bands of 16 rows, several
    # work items per box, whose outer items lie beyond 10 sigma of the compact components
    return synth.tiny(S=3, n_bands=2, size=72, side=61, seed=3)


@pytest.mark.parametrize("rows", [16, 8])
def test_culled_elbo_grad_hessian_and_hvp_match_oracle(B, O, synth, rows):
    f = wide_boxes(synth)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    plan = B.Plan(f)
    plan.set_launch(strip_rows=rows)
    wc = plan.work_counts(theta)
    b = np.asarray(f.boxes, np.int64)
    strips = int(np.sum(b[:, 4] * ((b[:, 3] + rows - 1) // rows)))
    assert wc["strips"] == strips and wc["visits"] == int(np.sum(b[:, 3] * b[:, 4]))
    live = wc["star_strips"] + wc["galaxy_strips"]
    say("rows", rows, "live Gaussians per strip %.2f of 45, pads %d" % (live / strips, wc["pad_strips"]))
    assert 0 < live < 45 * strips, "no culling on this field: the test would not exercise it"
    assert wc["pad_strips"] > 0 and wc["pad_visits"] > 0
    assert wc["star_visits"] <= 3 * wc["visits"] and wc["galaxy_visits"] <= 42 * wc["visits"]
    e, g = plan.elbo_grad(theta)
    e, g = e.cpu().numpy(), g.cpu().numpy()
    P = O.Problem(f)
    for s in range(f.n_src):
        val, gref, gabs = O.source_grad(P, s)
        within(np.array([e[s]]), np.array([val[0] + val[1]]), np.array([abs(val[2]) + abs(val[1])]),
               "rows %d elbo s=%d" % (rows, s))
        within(g[s, :27], gref, gabs, "rows %d grad s=%d" % (rows, s))
    H = plan.hessian(theta, np.arange(f.n_src)).cpu().numpy()
    for s in range(f.n_src):
        Href, Habs = O.source_hessian(P, s, with_abs=True)
        hessian_within(H[s], Href, Habs, "rows %d hessian s=%d" % (rows, s))
    # the dual-number passes cull too (one component at a time)
    v = np.random.default_rng(7 + rows).standard_normal(f.theta.shape)
    hv, g2 = plan.hvp(theta, torch.tensor(v, dtype=torch.float64, device="cuda"), with_grad=True)
    hv, g2 = hv.cpu().numpy(), g2.cpu().numpy()
    for s in range(f.n_src):
        ref, habs = O.source_hvp(P, s, v[s])
        within(hv[s, :27], ref, habs, "rows %d hvp s=%d" % (rows, s))
        _, gref, gabs = O.source_grad(P, s)
        within(g2[s, :27], gref, gabs, "rows %d hvp-grad s=%d" % (rows, s))


def test_work_counts_on_the_2000_source_field(B, synth):
    f = synth.field_2000src()
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    plan = B.Plan(f)
    wc = plan.work_counts(theta)
    b = np.asarray(f.boxes, np.int64)
    assert wc["strips"] == int(np.sum(b[:, 4] * ((b[:, 3] + 15) // 16)))
    assert wc["visits"] == int(np.sum(b[:, 3] * b[:, 4]))
    frac = (wc["star_strips"] + wc["galaxy_strips"]) / (45 * wc["strips"])
    say("live fraction %.3f" % frac)
    assert 0.5 < frac < 0.95
    # counts are properties of theta and the launch, not of earlier calls
    assert plan.work_counts(theta) == wc
