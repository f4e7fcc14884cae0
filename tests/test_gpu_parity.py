"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerance (per source s, parameter i): |gpu - oracle| <= 1e-9 |oracle| + 1e-12 G, where
G is the sum over visits of |per-visit term| reported by the oracle (FP64 summation
error of n terms is ~ log2(n) eps G, far below the floor).
"""
import sys

import numpy as np
import pytest

from conftest import hessian_within, newton_trajectory_parity

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
    """ELBO and gradient of the listed sources, batched (1) and plain (0), vs the oracle."""
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


def test_single_source(B, O, synth):
    f = synth.single_source()
    check_field(B, O, f, [0], name="single_source")


def test_region_16src_sampled(B, O, synth):
    f = synth.region_16src()
    check_field(B, O, f, [0, 7, 15], name="region_16src")


def test_plain_equals_batched_region_16src(B, synth):
    f = synth.region_16src()
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    plan = B.Plan(f)
    say("case region_16src plain-vs-batched")
    e1, g1 = plan.elbo_grad(theta, mode=1)
    e0, g0 = plan.elbo_grad(theta, mode=0)
    np.testing.assert_allclose(e0.cpu().numpy(), e1.cpu().numpy(), rtol=1e-11)
    ga = np.abs(g1.cpu().numpy()).max(axis=1, keepdims=True)
    assert np.all(np.abs(g0.cpu().numpy() - g1.cpu().numpy()) <= 1e-10 * np.abs(g1.cpu().numpy()) + 1e-12 * ga)


def test_hvp_matches_oracle(B, O, synth):
    f = synth.tiny(S=3, n_bands=2, size=17, side=11, seed=33)
    rng = np.random.default_rng(0)
    v = np.zeros((3, 48))
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
        Href, Habs = O.source_hessian(P, s, with_abs=True)
        hessian_within(H[k], Href, Habs, "hessian s=%d" % s)


@pytest.mark.parametrize("case", ["overlap", "masked-wcs-sky"])
@pytest.mark.parametrize("rows", [16, 4])
def test_hessian_closed_form_matches_tangent_passes_and_oracle(B, O, synth, case, rows):
    """The closed-form position / shape rows (default) and the five tangent passes give
    the same 27x27 Hessians, and both match the oracle's dual-number Hessian."""
    if case == "overlap":
        f = synth.tiny(S=4, n_bands=2, size=19, side=11, seed=35)
    else:
        f = synth.tiny(S=3, n_bands=3, size=21, side=13, seed=162, psf_xi=True, anisotropic_psf=True,
                       wcs=True, sky_map=True)
        rng = np.random.default_rng(9)
        f.x[rng.choice(f.x.size, 25, replace=False)] = np.nan
    th = f.theta.copy()
    th[:, 2] = np.linspace(0.2, 0.8, f.n_src)       # both galaxy profiles weigh in
    f.theta = th
    plan = B.Plan(f)
    plan.set_launch(strip_rows=rows)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    src = list(range(f.n_src))[::-1]
    say("case hessian modes", case, "rows", rows)
    H0 = plan.hessian(theta, src).cpu().numpy()
    plan.set_hessian_mode(1)
    H1 = plan.hessian(theta, src).cpu().numpy()
    plan.set_hessian_mode(0)
    P = O.Problem(f)
    for k, s in enumerate(src):
        scale = np.abs(H1[k]).max()
        np.testing.assert_allclose(H0[k], H1[k], rtol=1e-10, atol=1e-13 * scale)
        np.testing.assert_allclose(H0[k], H0[k].T, rtol=1e-10, atol=1e-13 * scale)
        Href, Habs = O.source_hessian(P, s, with_abs=True)
        hessian_within(H0[k], Href, Habs, "hessian %s rows %d s=%d" % (case, rows, s))


@pytest.mark.parametrize("rows", [16, 8, 4])
def test_second_order_on_multi_item_boxes(B, O, synth, rows):
    """Boxes of 35 x 35 pixels span several work items (2 at 16-row strips, 3 at 8, 5 at
    4), so the item sums of the pixel-level Hessian rows, the closed-form pass over items
    that start inside a box, the tangent passes and the Hessian-vector product all cross
    item boundaries: dense Hessians (both Hessian modes), HVPs and gradients against the
    oracle, per entry."""
    f = synth.tiny(S=3, n_bands=2, size=45, side=35, seed=204)
    th = f.theta.copy()
    th[:, 2] = [0.3, 0.6, 0.8]
    f.theta = th
    plan = B.Plan(f)
    plan.set_launch(strip_rows=rows)
    n_items = plan.info()["n_items"]
    assert n_items >= 2 * len(f.boxes)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    say("case multi-item second order rows", rows, "items", n_items)
    src = [2, 0, 1]
    H0 = plan.hessian(theta, src).cpu().numpy()
    plan.set_hessian_mode(1)
    H1 = plan.hessian(theta, src).cpu().numpy()
    plan.set_hessian_mode(0)
    rng = np.random.default_rng(rows)
    v = np.zeros((3, 48))
    v[:, :27] = rng.standard_normal((3, 27))
    hv, g = plan.hvp(theta, torch.tensor(v, device="cuda"), with_grad=True)
    hv, g = hv.cpu().numpy(), g.cpu().numpy()
    P = O.Problem(f)
    for k, s in enumerate(src):
        Href, Habs = O.source_hessian(P, s, with_abs=True)
        hessian_within(H0[k], Href, Habs, "closed-form hessian rows %d s=%d" % (rows, s))
        hessian_within(H1[k], Href, Habs, "tangent-pass hessian rows %d s=%d" % (rows, s))
        href, habs = O.source_hvp(P, s, v[s])
        within(hv[s, :27], href, habs, "multi-item hvp rows %d s=%d" % (rows, s))
        _, gref, gabs = O.source_grad(P, s)
        within(g[s, :27], gref, gabs, "multi-item grad rows %d s=%d" % (rows, s))


@pytest.fixture(scope="module")
def N():
    from oracle import newton
    return newton


def test_newton_on_multi_item_boxes(B, N, synth):
    """Newton iterations on boxes of two work items each (35 x 35 pixels, 16-row strips):
    every step within the derived one-step bound of the oracle's."""
    f = synth.tiny(S=3, n_bands=2, size=45, side=35, seed=203)
    say("case multi-item newton")
    newton_trajectory_parity(B, N, torch, f, [0, 1, 2], 3, say=say)


@pytest.mark.parametrize("mode", [1, 0])
def test_active_mask(B, O, synth, mode):
    """celeste_elbo / celeste_elbo_grad with an active mask: outputs of inactive sources are
    left as they were, active ones match the oracle (batched and plain)."""
    f = synth.tiny(S=6, n_bands=2, size=31, side=13, seed=211)
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    active = np.array([1, 0, 1, 1, 0, 0], np.uint8)
    act = torch.tensor(active, device="cuda")
    say("case active mask mode", mode)
    e = torch.full((6,), -7.5, dtype=torch.float64, device="cuda")
    g = torch.full((6, 48), 3.25, dtype=torch.float64, device="cuda")
    plan.elbo_grad(theta, mode=mode, active=act, elbo=e, grad=g)
    e2 = torch.full((6,), 11.0, dtype=torch.float64, device="cuda")
    plan.elbo(theta, mode=mode, active=act, out=e2)
    e, g, e2 = e.cpu().numpy(), g.cpu().numpy(), e2.cpu().numpy()
    for s in range(6):
        if not active[s]:
            assert e[s] == -7.5 and e2[s] == 11.0 and np.all(g[s] == 3.25), s
            continue
        ref, absum, gref, gabs = oracle_source(O, f, s)
        within(np.array([e[s]]), np.array([ref]), np.array([absum]), "active elbo_grad s=%d" % s)
        within(np.array([e2[s]]), np.array([ref]), np.array([absum]), "active elbo s=%d" % s)
        within(g[s, :27], gref, gabs, "active grad s=%d" % s)
        np.testing.assert_array_equal(g[s, 27:], 0.0)


def test_total_elbo(B, O, synth):
    f = synth.tiny(S=4, n_bands=2, size=21, side=9, seed=44)
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    say("case total elbo")
    t = plan.total_elbo(theta).cpu().numpy()[0]
    np.testing.assert_allclose(t, O.total_elbo(O.Problem(f)), rtol=1e-11)


LAUNCHES = [dict(chunk=64, waves_per_block=1, grid_blocks=256, dynamic=0, strip_rows=4, render_mode=0),
            dict(chunk=128, waves_per_block=2, grid_blocks=4096, dynamic=1, strip_rows=8, render_mode=1,
                 tile_h=16, tile_w=8),
            dict(chunk=1024, waves_per_block=4, grid_blocks=1024, dynamic=0, strip_rows=16, render_mode=0),
            dict(chunk=256, waves_per_block=4, grid_blocks=2048, dynamic=1, strip_rows=8, render_mode=1,
                 tile_h=16, tile_w=16),
            dict(chunk=64, waves_per_block=4, grid_blocks=0, dynamic=0, strip_rows=16, render_mode=2,
                 tile_h=16, tile_w=16),
            dict(chunk=128, waves_per_block=2, grid_blocks=512, dynamic=1, strip_rows=4, render_mode=2,
                 tile_h=4, tile_w=16),
            dict(chunk=64, waves_per_block=4, grid_blocks=1024, dynamic=0, strip_rows=16, render_mode=3),
            dict(chunk=192, waves_per_block=1, grid_blocks=300, dynamic=1, strip_rows=8, render_mode=3)]


def test_launch_configurations_agree(B, synth):
    f = synth.tiny(S=5, n_bands=3, size=40, side=23, seed=101)
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    e0, g0 = plan.elbo_grad(theta)
    e0, g0 = e0.cpu().numpy(), g0.cpu().numpy()
    gmax = np.abs(g0).max(axis=1, keepdims=True)
    for cfg in LAUNCHES:
        say("case launch", cfg)
        plan.set_launch(**cfg)
        e, g = plan.elbo_grad(theta)
        e, g = e.cpu().numpy(), g.cpu().numpy()
        np.testing.assert_allclose(e, e0, rtol=1e-12)
        assert np.all(np.abs(g - g0) <= 1e-11 * gmax)
        v = np.zeros((5, 48))
        v[:, :27] = 1.0
        hv = plan.hvp(theta, torch.tensor(v, device="cuda")).cpu().numpy()
        if cfg is LAUNCHES[0]:
            hv0 = hv
        else:
            assert np.all(np.abs(hv - hv0) <= 1e-11 * np.abs(hv0).max(axis=1, keepdims=True))


def test_graph_replays_match_eager(B, synth):
    f = synth.tiny(S=4, n_bands=2, size=30, side=15, seed=111)
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    e0, g0 = plan.elbo_grad(theta)
    e0, g0 = e0.clone(), g0.clone()
    plan.use_graph(True)
    elbo = torch.zeros_like(e0)
    grad = torch.zeros_like(g0)
    for rep in range(4):
        say("case graph replay", rep)
        elbo.fill_(0.0)
        grad.fill_(0.0)
        plan.elbo_grad(theta, elbo=elbo, grad=grad)
        torch.cuda.synchronize()
        assert torch.equal(elbo, e0) and torch.equal(grad, g0)
        x = torch.randn(1000, device="cuda").sum()      # unrelated eager work between replays
        torch.cuda.synchronize()
    plan.use_graph(False)


def test_two_runs_bitwise_equal(B, synth):
    f = synth.tiny(S=6, n_bands=2, size=40, side=21, seed=121)
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    a = [t.clone() for t in plan.elbo_grad(theta)]
    b = plan.elbo_grad(theta)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_source_without_boxes_and_ragged_boxes(B, O, synth):
    f = synth.tiny(S=3, n_bands=2, size=23, side=13, seed=131)
    # source 2 keeps no box: its ELBO is -KL only
    nb = int(f.patch_ptr[2])
    f.boxes = f.boxes[:nb]
    f.patch_ptr[3] = nb
    # ragged heights and widths
    f.boxes[0, 3] = 11
    f.boxes[1, 4] = 7
    check_field(B, O, f, range(3), name="ragged")


def test_degenerate_parameter_values(B, O, synth):
    """Parameters on the edges of their domain: frac_dev 0 and 1, a round galaxy, an angle
    many periods out, q next to 0 and 1, a galaxy far smaller than the PSF and one larger
    than its box.  ELBO, gradient (both modes), HVP and the closed-form Hessian."""
    f = synth.tiny(S=4, n_bands=2, size=21, side=11, seed=171)
    th = f.theta.copy()
    th[0, 2], th[0, 3] = 0.0, 1.0
    th[1, 2], th[1, 4] = 1.0, 7.0 * np.pi + 0.3
    th[2, 6], th[2, 5] = 1e-9, 0.02
    th[3, 6], th[3, 5] = 1.0 - 1e-9, 25.0
    f.theta = th
    plan, theta = check_field(B, O, f, range(4), name="degenerate")
    P = O.Problem(f)
    rng = np.random.default_rng(17)
    v = np.zeros((4, 48))
    v[:, :27] = rng.standard_normal((4, 27))
    say("case degenerate hvp / hessian")
    hv = plan.hvp(theta, torch.tensor(v, device="cuda")).cpu().numpy()
    H = plan.hessian(theta, [0, 1, 2, 3]).cpu().numpy()
    for s in range(4):
        ref, habs = O.source_hvp(P, s, v[s])
        within(hv[s, :27], ref, habs, "degenerate hvp s=%d" % s)
        Href, Habs = O.source_hessian(P, s, with_abs=True)
        hessian_within(H[s], Href, Habs, "hessian s=%d" % s)


def test_field_without_any_box(B, O, synth):
    """No source has a patch: every ELBO is -KL, the total ELBO is -sum KL, and the
    Hessian is the KL's."""
    f = synth.tiny(S=3, n_bands=2, size=15, side=9, seed=181)
    f.boxes = f.boxes[:0]
    f.patch_ptr = np.zeros_like(f.patch_ptr)
    plan, theta = check_field(B, O, f, range(3), name="no-box")
    P = O.Problem(f)
    say("case no-box hessian / total")
    H = plan.hessian(theta, [2, 1, 0]).cpu().numpy()
    for k, s in enumerate([2, 1, 0]):
        Href, Habs = O.source_hessian(P, s, with_abs=True)
        hessian_within(H[k], Href, Habs, "no-box hessian s=%d" % s)
    t = plan.total_elbo(theta).cpu().numpy()[0]
    np.testing.assert_allclose(t, O.total_elbo(P), rtol=1e-12)


def test_single_pixel_and_whole_image_boxes(B, O, synth):
    """1 x 1 boxes in opposite image corners and a box covering a whole image."""
    f = synth.tiny(S=3, n_bands=2, size=17, side=9, seed=191)
    H_, W_ = 17, 17
    b = f.boxes.copy()
    for k in range(len(b)):
        src = int(np.searchsorted(f.patch_ptr, k, side="right") - 1)
        if src == 0:
            b[k, 1:] = (0, 0, 1, 1) if b[k, 0] == 0 else (H_ - 1, W_ - 1, 1, 1)
        elif src == 1:
            b[k, 1:] = (0, 0, H_, W_)
    f.boxes = b
    plan, theta = check_field(B, O, f, range(3), name="corner-boxes")
    P = O.Problem(f)
    say("case corner-boxes hessian")
    H = plan.hessian(theta, [0, 1, 2]).cpu().numpy()
    for s in range(3):
        Href, Habs = O.source_hessian(P, s, with_abs=True)
        hessian_within(H[s], Href, Habs, "hessian s=%d" % s)


def test_masked_pixels(B, O, synth):
    f = synth.tiny(S=2, n_bands=2, size=19, side=13, seed=141)
    rng = np.random.default_rng(5)
    f.x[rng.choice(f.x.size, 20, replace=False)] = np.nan
    check_field(B, O, f, range(2), name="masked")


def test_field_2000src_full_size_sampled(B, O, synth):
    """Full field at the benchmark's launch configuration (plan default, graph replay), then
    at the autotuned one."""
    f = synth.field_2000src()
    plan = B.Plan(f)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    P = O.Problem(f)
    refs = {s: O.source_grad(P, s) for s in [0, 517, 1999]}
    say("case field_2000src full plain")
    e, g = plan.elbo_grad(theta, mode=B.CELESTE_PLAIN)
    e, g = e.cpu().numpy(), g.cpu().numpy()
    for s, (val, gref, gabs) in refs.items():
        within(np.array([e[s]]), np.array([val[0] + val[1]]), np.array([abs(val[2]) + abs(val[1])]), "c2 plain elbo")
        within(g[s, :27], gref, gabs, "c2 plain grad s=%d" % s)
    for tuned in (False, True):
        if tuned:
            plan.autotune(theta, reps=1)
        plan.use_graph(True)
        say("case field_2000src full", "autotuned" if tuned else "default", plan.info())
        e, g = plan.elbo_grad(theta)
        e, g = e.cpu().numpy(), g.cpu().numpy()
        for s, (val, gref, gabs) in refs.items():
            within(np.array([e[s]]), np.array([val[0] + val[1]]), np.array([abs(val[2]) + abs(val[1])]), "c2 elbo")
            within(g[s, :27], gref, gabs, "c2 grad s=%d" % s)
        plan.use_graph(False)


def test_table_exp_accuracy(B):
    """The strip kernels' table-driven exp against the host libm exp, in ulps."""
    rng = np.random.default_rng(9)
    x = np.concatenate([rng.uniform(-745.0, 709.0, 200000), rng.uniform(-40.0, 3.0, 200000),
                        rng.uniform(-1e-3, 1e-3, 10000), [0.0, -0.0, 1.0, -1.0, 700.0, -700.0, -744.0, 709.0],
                        np.log(2.0) / 64 * np.arange(-200, 200)])
    say("case table exp", x.size)
    y = B.debug_math(B.FN_EXP, torch.tensor(x, device="cuda")).cpu().numpy()
    ref = np.exp(x)
    normal = ref >= 2.2250738585072014e-308
    ulp = np.spacing(ref[normal])
    err = np.abs(y[normal] - ref[normal]) / ulp
    assert err.max() <= 4.0, err.max()
    assert np.all(np.abs(y[~normal] - ref[~normal]) <= 4 * 5e-324)


def test_table_log_and_reciprocal_accuracy(B):
    """The pixel term's table-driven log and Newton reciprocal against the host libm."""
    rng = np.random.default_rng(10)
    x = np.concatenate([np.exp(rng.uniform(-700.0, 700.0, 200000)), rng.uniform(50.0, 1e5, 200000),
                        rng.uniform(0.25, 4.0, 100000), [1.0, 2.0, 0.5, 1e-300, 1e300, 3.0, 7.0],
                        0.5 + (np.arange(128) + 0.5) / 256.0, 0.5 + np.arange(129) / 256.0])
    say("case table log / rcp", x.size)
    xd = torch.tensor(x, device="cuda")
    lg = B.debug_math(B.FN_LOG, xd).cpu().numpy()
    ref = np.log(x)
    # a few ulps relative; near x = 1 the m ln2 and log F terms cancel: a few 1e-16 absolute
    err = np.abs(lg - ref)
    assert np.all(err <= 4 * np.spacing(np.abs(ref)) + 4e-16), (err / np.maximum(np.spacing(np.abs(ref)), 1e-300)).max()
    far = np.abs(x - 1.0) > 0.5
    assert (err[far] / np.spacing(np.abs(ref[far]))).max() <= 4.0
    rc = B.debug_math(B.FN_RCP, xd).cpu().numpy()
    ok = np.abs(x) < 1e307
    assert np.all(np.abs(rc[ok] - 1.0 / x[ok]) <= 1.0 * np.spacing(1.0 / x[ok]))


def test_astrometry_and_sky_maps(B, O, synth):
    """Rotated, scaled and sheared astrometry plus per-pixel sky maps: ELBO and gradient
    (batched and plain), HVP, dense Hessian and total ELBO against the oracle."""
    f = synth.tiny(S=3, n_bands=3, size=21, side=13, seed=161, psf_xi=True, anisotropic_psf=True,
                   wcs=True, sky_map=True)
    f.img_origin[1] = [0.6, -0.4]
    plan, theta = check_field(B, O, f, range(3), name="wcs-sky")
    rng = np.random.default_rng(3)
    v = np.zeros((3, 48))
    v[:, :27] = rng.standard_normal((3, 27))
    say("case wcs-sky hvp / hessian / total")
    hv = plan.hvp(theta, torch.tensor(v, device="cuda")).cpu().numpy()
    P = O.Problem(f)
    for s in range(3):
        ref, habs = O.source_hvp(P, s, v[s])
        within(hv[s, :27], ref, habs, "wcs-sky hvp s=%d" % s)
    H = plan.hessian(theta, [2, 0]).cpu().numpy()
    for k, s in enumerate([2, 0]):
        Href, Habs = O.source_hessian(P, s, with_abs=True)
        hessian_within(H[k], Href, Habs, "wcs-sky hessian s=%d" % s)
    t = plan.total_elbo(theta).cpu().numpy()[0]
    np.testing.assert_allclose(t, O.total_elbo(P), rtol=1e-11)
