"""GPU trust-region Newton and block-coordinate sweeps against the oracle."""
import sys

import numpy as np
import pytest

from conftest import newton_trajectory_parity, sweep_batch_parity

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


def boxes_conflict(f, s, t):
    for bs in f.boxes[f.patch_ptr[s]:f.patch_ptr[s + 1]]:
        for bt in f.boxes[f.patch_ptr[t]:f.patch_ptr[t + 1]]:
            if bs[0] != bt[0]:
                continue
            if bs[1] < bt[1] + bt[3] and bt[1] < bs[1] + bs[3] and bs[2] < bt[2] + bt[4] and bt[2] < bs[2] + bs[4]:
                return True
    return False


@pytest.mark.parametrize("steps", [1, 4])
def test_newton_matches_oracle_overlapping_sources(B, N, synth, steps):
    """Three overlapping sources optimised together (each with the others at their entry
    values): every step of the device's run within the derived one-step bound of the
    oracle's step from the device's previous iterate, same radius, ELBO_s to 1e-9."""
    f = synth.tiny(S=3, n_bands=2, size=17, side=11, seed=12)
    say("case newton steps", steps)
    worst = newton_trajectory_parity(B, N, torch, f, [0, 1, 2], steps, say=say)
    say("  observed max |diff| / bound", worst)


@pytest.mark.parametrize("gtol", [1.0, 10.0, 1e30])
def test_newton_gradient_stop_matches_oracle(B, N, synth, gtol):
    """A source stops once its largest unconstrained gradient entry is below gtol.  On this
    field with 6 iterations, gtol 1 stops sources 1 and 2 early but not source 0, gtol 10
    stops all three at different iterations, and gtol 1e30 stops every source before its
    first step (no gradient within 10% of either threshold, so rounding cannot move a
    stop).  Every step matches the oracle's step with the same rule (derived bound; a
    stopped source keeps its parameters exactly)."""
    f = synth.tiny(S=3, n_bands=2, size=17, side=11, seed=12)
    say("case newton gtol", gtol)
    newton_trajectory_parity(B, N, torch, f, [0, 1, 2], 6, gtol=gtol, say=say)
    if gtol == 1e30:
        plan = B.Plan(f)
        theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
        _, radius = plan.newton(theta, [0, 1, 2], 6, params=B.tr_params(gtol=gtol))
        np.testing.assert_array_equal(theta.cpu().numpy(), f.theta)
        np.testing.assert_array_equal(radius.cpu().numpy(), 1.0)


def test_newton_stored_and_evaluated_backgrounds_agree(B, synth):
    """Newton iterations with the strip render (backgrounds summed from every box's stored
    own values) and with the tile render (backgrounds evaluated from the tables) reach the
    same parameters and ELBO."""
    f = synth.tiny(S=6, n_bands=2, size=29, side=11, seed=78)
    out = []
    for launch in (dict(), dict(render_mode=1)):
        plan = B.Plan(f)
        if launch:
            plan.set_launch(**launch)
        theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
        say("case newton backgrounds", launch)
        elbo, radius = plan.newton(theta, list(range(6)), 4)
        out.append((theta.cpu().numpy(), elbo.cpu().numpy(), radius.cpu().numpy()))
    (t0, e0, r0), (t1, e1, r1) = out
    assert np.all(np.abs(t0 - t1) <= 1e-8 * (1.0 + np.abs(t1))), np.max(np.abs(t0 - t1))
    np.testing.assert_allclose(e0, e1, rtol=1e-12)
    np.testing.assert_array_equal(r0, r1)


def test_newton_same_with_either_hessian_mode(B, synth):
    """Newton iterations with the closed-form Hessian rows (default) and with the tangent
    passes reach the same parameters."""
    f = synth.tiny(S=5, n_bands=2, size=23, side=11, seed=13)
    out = []
    for mode in (0, 1):
        plan = B.Plan(f)
        plan.set_hessian_mode(mode)
        theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
        say("case newton hessian mode", mode)
        plan.newton(theta, list(range(5)), 4)
        out.append(theta.cpu().numpy())
    scale = 1.0 + np.abs(out[1])
    assert np.all(np.abs(out[0] - out[1]) <= 1e-8 * scale), np.max(np.abs(out[0] - out[1]) / scale)


def test_conflict_free_batch_equals_one_at_a_time(B, synth):
    f = synth.tiny(S=4, n_bands=2, size=31, side=9, seed=61)
    plan = B.Plan(f)
    ptr, src = plan.color_batches(seed=3)
    batch = src[ptr[0]:ptr[1]]
    assert len(batch) >= 2
    for i in range(len(batch)):
        for j in range(i + 1, len(batch)):
            assert not boxes_conflict(f, batch[i], batch[j])
    say("case batch vs sequential", batch.tolist())
    th1 = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    plan.newton(th1, batch, 3)
    th2 = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    for s in batch:
        plan.newton(th2, [int(s)], 3)
    assert torch.max(torch.abs(th1 - th2)).item() <= 1e-12 * torch.max(torch.abs(th1)).item()


def test_sweep_trajectory(B, N, O, synth):
    f = synth.tiny(S=4, n_bands=2, size=25, side=9, seed=71)
    plan = B.Plan(f)
    ptr, src = plan.color_batches(seed=1)
    for b in range(len(ptr) - 1):
        mem = src[ptr[b]:ptr[b + 1]]
        for i in range(len(mem)):
            for j in range(i + 1, len(mem)):
                assert not boxes_conflict(f, mem[i], mem[j])
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    say("case sweep", ptr.tolist())
    params = B.tr_params(newton_steps=3)
    trace = plan.sweep(theta, ptr, src, 2, params).cpu().numpy()
    assert np.all(np.diff(trace) >= -1e-9 * np.abs(trace[:-1]))
    np.testing.assert_allclose(trace[0], O.total_elbo(O.Problem(f)), rtol=1e-11)
    th_gpu = theta.cpu().numpy()
    np.testing.assert_allclose(trace[-1], O.total_elbo(O.Problem(f, th_gpu)), rtol=1e-11)
    # one sweep with one Newton step per batch visit, batch by batch against the oracle
    say("case sweep per-batch parity")
    sweep_batch_parity(B, N, torch, f, ptr, src, say=say)


def test_conflict_graph_matches_oracle(B, synth):
    from oracle import schedule as Sch
    for f in (synth.tiny(S=8, n_bands=2, size=33, side=9, seed=73), synth.region_16src()):
        say("case conflict graph", f.n_src)
        plan = B.Plan(f)
        ptr, adj = plan.conflict_graph()
        assert Sch.adjacency_sets(ptr, adj) == Sch.conflict_graph(f)
        for s in range(f.n_src):
            assert np.all(np.diff(adj[ptr[s]:ptr[s + 1]]) > 0)   # sorted, no repeats


def test_cyclades_epoch_equals_serial_bca(B, N, O, synth):
    """One epoch over the Cyclades rounds (Section IV-D) gives the parameters of serial
    block coordinate ascent in the sampling order, replayed on the oracle one source at
    a time with every other source at its current value."""
    from oracle import schedule as Sch
    f = synth.tiny(S=8, n_bands=2, size=33, side=9, seed=73)
    plan = B.Plan(f)
    bp, bs, nc, order = plan.cyclades_batches(seed=5, sample_size=5)
    rounds = [bs[bp[b]:bp[b + 1]].tolist() for b in range(len(bp) - 1)]
    assert (rounds, nc) == Sch.cyclades_rounds(Sch.conflict_graph(f), order, 5)
    assert max(len(r) for r in rounds) >= 2 and len(rounds) > 2   # side by side and serial both occur
    say("case cyclades epoch", order.tolist(), rounds)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    params = B.tr_params(newton_steps=1)
    trace = plan.sweep(theta, bp, bs, 1, params).cpu().numpy()
    t1 = theta.cpu().numpy()
    np.testing.assert_array_equal(t1[:, 27:], 0.0)
    np.testing.assert_allclose(trace[0], O.total_elbo(O.Problem(f)), rtol=1e-11)
    np.testing.assert_allclose(trace[1], O.total_elbo(O.Problem(f, t1)), rtol=1e-11)
    assert trace[1] >= trace[0]
    # round by round: each member's step from the device's state before its round is the
    # oracle's step from that state; members of a round share no pixel, and the rounds are
    # the oracle's schedule (checked above), so the epoch is serial block coordinate ascent
    # in the sampling order
    say("case cyclades per-round parity")
    last, _ = sweep_batch_parity(B, N, torch, f, bp, bs, say=say)
    np.testing.assert_array_equal(last, t1)


def test_sweep_stored_and_evaluated_backgrounds_agree(B, synth):
    """A sweep with the strip render (batch backgrounds summed from stored values) and one
    with the tile render at another strip height (backgrounds evaluated from the tables)
    reach the same parameters and ELBO trace."""
    f = synth.tiny(S=6, n_bands=2, size=29, side=11, seed=77)
    out = []
    for launch in (dict(), dict(strip_rows=8, render_mode=1)):
        plan = B.Plan(f)
        if launch:
            plan.set_launch(**launch)
        ptr, src = plan.color_batches(seed=2)
        theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
        say("case sweep backgrounds", launch)
        trace = plan.sweep(theta, ptr, src, 2, B.tr_params(newton_steps=3)).cpu().numpy()
        out.append((theta.cpu().numpy(), trace))
    (t0, e0), (t1, e1) = out
    assert np.all(np.abs(t0 - t1) <= 1e-8 * (1.0 + np.abs(t1))), np.max(np.abs(t0 - t1))
    np.testing.assert_allclose(e0, e1, rtol=1e-12)


def test_sweep_rejects_conflicting_batch(B, synth):
    f = synth.tiny(S=3, n_bands=1, size=15, side=11, seed=81)
    plan = B.Plan(f)
    assert boxes_conflict(f, 0, 1)
    theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    with pytest.raises(B.CelesteError) as e:
        plan.sweep(theta, np.array([0, 2]), np.array([0, 1]), 1)
    assert e.value.code == B.CELESTE_ECONFLICT
    np.testing.assert_array_equal(theta.cpu().numpy(), f.theta)


def test_domain_error_leaves_outputs(B, synth):
    f = synth.tiny(S=2, n_bands=1, size=15, side=9, seed=91)
    plan = B.Plan(f)
    bad = f.theta.copy()
    bad[1, 6] = 1.5          # probability out of (0, 1)
    theta = torch.tensor(bad, dtype=torch.float64, device="cuda")
    elbo = torch.full((2,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(B.CelesteError) as e:
        plan.elbo(theta, out=elbo)
    assert e.value.code == B.CELESTE_EDOMAIN
    assert torch.all(elbo == 7.0)


def test_newton_with_astrometry_and_sky_maps(B, N, synth):
    f = synth.tiny(S=3, n_bands=2, size=19, side=13, seed=171, wcs=True, sky_map=True)
    say("case newton wcs-sky")
    newton_trajectory_parity(B, N, torch, f, [0, 1, 2], 2, say=say)


def test_plan_rejects_bad_image_metadata(B, synth):
    """A sky map with a non-positive entry or a singular astrometry is refused at plan
    creation (host check of the map, before anything else is allocated)."""
    f = synth.tiny(S=2, n_bands=2, size=15, side=9, seed=181, wcs=True, sky_map=True)
    bad = f.sky_map.copy()
    bad[37] = 0.0
    g = type(f)(**{**f.__dict__, "sky_map": bad})
    with pytest.raises(B.CelesteError) as e:
        B.Plan(g)
    assert e.value.code == B.CELESTE_EINVAL
    w = f.img_wcs.copy()
    w[1] = [[1.0, 2.0], [0.5, 1.0]]
    h = type(f)(**{**f.__dict__, "img_wcs": w})
    with pytest.raises(B.CelesteError) as e:
        B.Plan(h)
    assert e.value.code == B.CELESTE_EINVAL
    B.Plan(f)


@pytest.mark.parametrize("schedule", ["colour", "cyclades"])
def test_sweep_graph_replays_match_eager(B, synth, schedule):
    """Sweeps replayed from a captured HIP graph (celeste_plan_use_graph) give bitwise the
    parameters and ELBO trace of the eager sweeps, over several replays in one call and
    over two calls with unrelated eager work and synchronisations in between."""
    f = synth.tiny(S=8, n_bands=2, size=33, side=9, seed=73)
    eager = B.Plan(f)
    if schedule == "colour":
        ptr, src = eager.color_batches(seed=3)
    else:
        ptr, src, _, _ = eager.cyclades_batches(seed=5, sample_size=5)
    params = B.tr_params(newton_steps=2)
    th_e = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    tr_e = [eager.sweep(th_e, ptr, src, 3, params).clone()]
    tr_e.append(eager.sweep(th_e, ptr, src, 2, params).clone())
    graph = B.Plan(f)
    graph.use_graph(True)
    th_g = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    say("case sweep graph", schedule, len(ptr) - 1, "batches")
    tr_g = [graph.sweep(th_g, ptr, src, 3, params).clone()]
    torch.cuda.synchronize()
    x = torch.randn(4096, device="cuda").sum()       # unrelated eager work between calls
    torch.cuda.synchronize()
    tr_g.append(graph.sweep(th_g, ptr, src, 2, params).clone())
    torch.cuda.synchronize()
    for a, b in zip(tr_e, tr_g):
        assert torch.equal(a, b), (a, b)
    assert torch.equal(th_e, th_g)


def test_newton_one_source_equals_its_part_of_a_batch(B, synth):
    """Newton on one listed source (its backgrounds from the stored values of its neighbour
    boxes only) gives bitwise the parameters, ELBO and radius that source reaches when every
    source is listed (each listed source sees the others at their entry values)."""
    f = synth.tiny(S=10, n_bands=2, size=60, side=11, seed=91)
    plan = B.Plan(f)
    th_all = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
    e_all, r_all = plan.newton(th_all, list(range(10)), 3)
    for s in (0, 4, 9):
        th = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
        say("case newton one source", s)
        e1, r1 = plan.newton(th, [s], 3)
        assert torch.equal(th[s], th_all[s]) and e1[s] == e_all[s] and r1[s] == r_all[s], s
        others = [t for t in range(10) if t != s]
        np.testing.assert_array_equal(th.cpu().numpy()[others], f.theta[others])
        # a Hessian call on a fresh plan (no tables left by an earlier call) for one source
        # and for all of them
        fresh = B.Plan(f)
        H1 = fresh.hessian(th, [s])
        Ha = B.Plan(f).hessian(th, list(range(10)))
        assert torch.equal(H1[0], Ha[s]), s
