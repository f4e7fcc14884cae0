"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerance (per source s, parameter i): |gpu - oracle| <= 1e-9 |oracle| + 1e-12 G, where
G is the sum over visits of |per-visit term| reported by the oracle (FP64 summation
error of n terms is ~ log2(n) eps G, far below the floor).
"""
import sys

import numpy as np
import pytest

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
    assert not bad.any(), "%s: max err/bound %.3g at %s (got %s ref %s)" % (
        what, (err / np.maximum(bound, 1e-300)).max(), np.argwhere(bad)[:5].tolist(),
        got[bad][:3], ref[bad][:3])
    return float((err / np.maximum(np.abs(ref), 1e-300)).max())


def oracle_source(O, f, s):
    P = O.Problem(f)
    val, g, ga = O.source_grad(P, s)
    return val[0] + val[1], abs(val[2]) + abs(val[1]), g, ga


def check_field(B, O, f, sources, modes=(1, 0), name=""):
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    plan = B.Plan(f)
    for mode in modes:
        say("case", name, "mode", mode)
        e, g = plan.elbo_grad(theta, mode=mode)
        e2 = plan.elbo(theta, mode=mode)
        e, g, e2 = e.cpu().numpy(), g.cpu().numpy(), e2.cpu().numpy()
        np.testing.assert_array_equal(g[:, 27:], 0.0)
        for s in sources:
            ref, absum, gref, gabs = oracle_source(O, f, s)
            within(np.array([e[s]]), np.array([ref]), np.array([absum]), "%s elbo_grad value s=%d" % (name, s))
            within(np.array([e2[s]]), np.array([ref]), np.array([absum]), "%s elbo value s=%d" % (name, s))
            within(g[s, :27], gref, gabs, "%s grad s=%d mode=%d" % (name, s, mode))
    return plan, theta


def test_tiny_overlapping(B, O, synth):
    f = synth.tiny(S=3, n_bands=3, size=17, side=11, seed=21)
    check_field(B, O, f, range(3), name="tiny3")


def test_tiny_general_psf_and_origin(B, O, synth):
    f = synth.tiny(S=2, n_bands=2, size=19, side=13, seed=5, psf_xi=True, anisotropic_psf=True)
    f.img_origin[1] = [0.37, -0.81]
    f.flags = synth.FLAG_INCLUDE_KL | synth.FLAG_INCLUDE_LGAMMA
    check_field(B, O, f, range(2), name="tiny-psf")


def test_config0(B, O, synth):
    f = synth.make_config(0)
    check_field(B, O, f, [0], name="config0")


def test_config1_sampled(B, O, synth):
    f = synth.make_config(1)
    check_field(B, O, f, [0, 7, 15], name="config1")


def test_plain_equals_batched_config1(B, synth):
    f = synth.make_config(1)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    plan = B.Plan(f)
    say("case config1 plain-vs-batched")
    e1, g1 = plan.elbo_grad(theta, mode=1)
    e0, g0 = plan.elbo_grad(theta, mode=0)
    np.testing.assert_allclose(e0.cpu().numpy(), e1.cpu().numpy(), rtol=1e-11)
    ga = np.abs(g1.cpu().numpy()).max(axis=1, keepdims=True)
    assert np.all(np.abs(g0.cpu().numpy() - g1.cpu().numpy()) <= 1e-10 * np.abs(g1.cpu().numpy()) + 1e-12 * ga)


def test_hvp_matches_oracle(B, O, synth):
    f = synth.tiny(S=3, n_bands=2, size=17, side=11, seed=33)
    rng = np.random.default_rng(0)
    v = np.zeros((3, 32))
    v[:, :27] = rng.standard_normal((3, 27))
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    say("case hvp tiny")
    hv, g = plan.hvp(theta, torch.tensor(v, device="cuda"), with_grad=True)
    hv, g = hv.cpu().numpy(), g.cpu().numpy()
    P = O.Problem(f)
    for s in range(3):
        ref, habs = O.source_hvp(P, s, v[s])
        within(hv[s, :27], ref, habs, "hvp s=%d" % s)
        _, gref, gabs = O.source_grad(P, s)
        within(g[s, :27], gref, gabs, "hvp-grad s=%d" % s)


def test_hessian_matches_oracle(B, O, synth):
    f = synth.tiny(S=2, n_bands=2, size=15, side=11, seed=34)
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    say("case hessian tiny")
    H = plan.hessian(theta, [1, 0]).cpu().numpy()
    P = O.Problem(f)
    for k, s in enumerate([1, 0]):
        Href = O.source_hessian(P, s)
        scale = np.abs(Href).max()
        np.testing.assert_allclose(H[k], Href, rtol=1e-8, atol=1e-11 * scale)


def test_total_elbo(B, O, synth):
    f = synth.tiny(S=4, n_bands=2, size=21, side=9, seed=44)
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    say("case total elbo")
    t = plan.total_elbo(theta).cpu().numpy()[0]
    np.testing.assert_allclose(t, O.total_elbo(O.Problem(f)), rtol=1e-11)
