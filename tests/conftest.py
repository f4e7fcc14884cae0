import copy
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def synth():
    from paper_1801_10277_amd import synth as s
    return s


@pytest.fixture(scope="session")
def O():
    from oracle import oracle as o
    o.build()
    return o


def clone(f):
    return copy.deepcopy(f)


def _boxes_meet(a, b):
    return (a[0] == b[0] and a[1] < b[1] + b[3] and b[1] < a[1] + a[3] and a[2] < b[2] + b[4]
            and b[2] < a[2] + a[4])


def neighbourhood(f, s, theta=None):
    """Source s with every source that has a box meeting one of s's boxes (same image), in
    their original order, over the same images: (sub-field, index of s in it).  Pixels of
    s's boxes see exactly these sources, so s's ELBO, gradient and Newton steps (others
    fixed) are those of the full field."""
    th = f.theta if theta is None else theta
    ptr = np.asarray(f.patch_ptr)
    mine = f.boxes[ptr[s]:ptr[s + 1]]
    keep = []
    for t in range(f.n_src):
        if t == s or any(_boxes_meet(a, b) for a in mine for b in f.boxes[ptr[t]:ptr[t + 1]]):
            keep.append(t)
    g = copy.copy(f)
    g.theta = np.ascontiguousarray(th[keep])
    g.boxes = np.ascontiguousarray(np.concatenate([f.boxes[ptr[t]:ptr[t + 1]] for t in keep]))
    counts = [ptr[t + 1] - ptr[t] for t in keep]
    g.patch_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    g.truth = {}
    return g, keep.index(s)


def single_source(synth, size=41, side=None, star=True, q=None, seed=3, psf_sigmas=None,
                  psf_weights=None, center=None, shape=None, sky=150.0, n_bands=1, band0=2,
                  r_var=0.01, c_var=0.01):
    """A one-source field built by hand: square image(s), box = whole image by default."""
    f = synth.tiny(S=1, n_bands=n_bands, size=size, side=size if side is None else side,
                   seed=seed)
    f.flags = synth.FLAG_INCLUDE_KL
    f.img_band = np.arange(band0, band0 + n_bands, dtype=np.int32) % 5
    f.img_sky[:] = sky
    if psf_sigmas is not None:
        f.img_psf[:, :, 3] = np.asarray(psf_sigmas) ** 2
        f.img_psf[:, :, 5] = np.asarray(psf_sigmas) ** 2
        f.img_psf[:, :, 4] = 0.0
        f.img_psf[:, :, 1:3] = 0.0
    if psf_weights is not None:
        f.img_psf[:, :, 0] = psf_weights
    c = (size - 1) / 2.0 if center is None else center
    f.theta[0, 0] = c
    f.theta[0, 1] = c
    if shape is not None:
        f.theta[0, 2:6] = shape
    if q is not None:
        f.theta[0, 6] = q
    for base in (7, 17):
        f.theta[0, base + 1] = r_var
        f.theta[0, base + 6:base + 10] = c_var
    if side is None:
        f.boxes = np.array([[n, 0, 0, size, size] for n in range(n_bands)], np.int32)
    else:
        cc = int(np.floor(c + 0.5))
        h = side // 2
        r0, r1 = max(cc - h, 0), min(cc + h + 1, size)
        f.boxes = np.array([[n, r0, r0, r1 - r0, r1 - r0] for n in range(n_bands)], np.int32)
    f.patch_ptr = np.array([0, n_bands], np.int32)
    return f


# ---------------------------------------------------------------- derived tolerances
REL = 1e-9      # relative gate of the parity tests (per value, gradient and HVP entry)
FLOOR = 1e-12   # times the sum of |per-visit terms|: FP64 summation error ~ log2(n) eps G


def hessian_within(H, Href, Habs, what):
    """Per-element bound of a dense Hessian, the gradient's gate applied entry by entry:
    |H - Href| <= 1e-9 |Href| + 1e-12 Habs (Habs: the oracle's sum of |per-visit terms|).
    Returns the largest pure relative error."""
    err = np.abs(H - Href)
    bound = REL * np.abs(Href) + FLOOR * Habs
    bad = err > bound
    assert not bad.any(), "%s: max err/bound %.3g at %s" % (
        what, (err / np.maximum(bound, 1e-300)).max(), np.argwhere(bad)[:5].tolist())
    return float((err / np.maximum(np.abs(Href), 1e-300)).max())


def newton_step_bound(N, f, theta, s, radius, gtol=1e-8):
    """One trust-region step of source s from `theta` (every other source fixed) with radius
    `radius` on the oracle, and a first-order bound on |theta_gpu - theta_oracle| after it,
    given that the device's gradient and Hessian meet the per-entry gates (1e-9 relative +
    1e-12 of the sum of |per-visit terms|).

    In unconstrained coordinates the step solves (B + mu I) p = -g with |p| = R when mu > 0.
    Perturbing g and B by dg, dB (and mu so that |p| stays R) moves p by
    dp = -P M^-1 (dg + dB p), M = B + mu I, P = I - M^-1 p p^T / (p^T M^-1 p) (P = I for an
    interior step), so |dp| <= |P M^-1| (|dg| + |dB|_F |p|); both solves stop the secular
    equation at |p| within 1e-13 R, which adds 2e-13 R |P M^-1| |M|.  theta_i moves by at
    most |row i of the Jacobian of theta(eta) at the trial point| |dp|.  A source that stops before stepping keeps theta exactly
    (bound 0).  Returns (bound[27], oracle row, oracle ELBO_s, oracle radius)."""
    rec = []
    row, fend, R = N.newton_steps(f, theta, s, 1, radius0=radius, gtol=gtol, record=rec)
    npar = len(row)
    if not rec:
        return np.zeros(npar), row, fend, R
    r0 = rec[0]
    g, gabs, H, Habs, B, p = r0["grad"], r0["gabs"], r0["hess"], r0["habs"], r0["B"], r0["step"]
    eta, J, curvature = N.transform(theta[s, :npar], npar)
    dg = REL * np.abs(g) + FLOOR * gabs
    dH = REL * np.abs(H) + FLOOR * Habs
    dgm = np.abs(J).T @ dg
    dB = np.abs(J).T @ dH @ np.abs(J) + curvature(dg, absolute=True)
    m = len(p)
    pn = np.linalg.norm(p)
    res = -r0["g_eta"] - B @ p
    mu = max(0.0, (res @ p) / (p @ p)) if pn > 0 else 0.0
    M = B + mu * np.eye(m)
    Minv = np.linalg.inv(M)
    if mu > 0:
        Mp = Minv @ p
        Proj = np.eye(m) - np.outer(Mp, p) / (p @ Mp)
    else:
        Proj = np.eye(m)
    PM = np.linalg.norm(Proj @ Minv, 2)
    dp = PM * (np.linalg.norm(dgm) + np.linalg.norm(dB) * pn) + 2e-13 * radius * PM * np.linalg.norm(M, 2)
    th1 = N.row_from_eta(eta + p, npar)
    _, J1, _ = N.transform(th1, npar)
    bound = np.linalg.norm(J1, axis=1) * dp + 4e-16 * np.abs(th1)
    return bound, row, fend, R


def newton_trajectory_parity(B, N, torch, f, srcs, steps, gtol=1e-8, say=print):
    """Per-step parity of a Newton run (each listed source optimised with every other source
    at its entry value): the device's k-step runs give its iterates theta_k (a k-step run
    takes the same first k steps as a longer one); for every k and listed source, the
    oracle takes one step from the device's theta_{k-1} and radius_{k-1}, and the device's
    theta_k must lie within newton_step_bound of it, with the same radius and ELBO_s to
    1e-9.  Returns the largest |difference| / bound seen (0 when every step was exact)."""
    plan = B.Plan(f)
    params = B.tr_params(gtol=gtol)
    prev_th = f.theta.copy()
    prev_R = np.full(f.n_src, params.radius0)
    worst = 0.0
    for k in range(1, steps + 1):
        theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
        elbo, radius = plan.newton(theta, np.asarray(srcs, np.int32), k, params=params)
        thk, ek, Rk = theta.cpu().numpy(), elbo.cpu().numpy(), radius.cpu().numpy()
        np.testing.assert_array_equal(np.delete(thk, srcs, axis=0), np.delete(f.theta, srcs, axis=0))
        for s in srcs:
            base = f.theta.copy()
            base[s] = prev_th[s]
            bound, row, fend, R = newton_step_bound(N, f, base, s, prev_R[s], gtol=gtol)
            diff = np.abs(thk[s, :len(row)] - row)
            assert np.all(diff <= bound), (k, s, (diff / np.maximum(bound, 1e-300)).max())
            worst = max(worst, float(np.max(np.where(bound > 0, diff / np.maximum(bound, 1e-300), 0.0))))
            assert Rk[s] == R, (k, s, Rk[s], R)
            np.testing.assert_allclose(ek[s], fend, rtol=1e-9)
        say("  newton step", k, "worst |diff| / bound %.3g" % worst)
        prev_th, prev_R = thk, Rk
    return worst


def sweep_batch_parity(B, N, torch, f, ptr, src, say=print):
    """Per-step parity of one block-coordinate-ascent sweep with one Newton step per batch
    visit: the device's state after batch b comes from a sweep over the schedule's first
    b + 1 batches; every member of batch b must then lie within newton_step_bound of the
    oracle's step from the device's state after batch b - 1 (every other source at its
    current value), non-members must be unchanged.  Returns the largest |diff| / bound."""
    plan = B.Plan(f)
    params = B.tr_params(newton_steps=1)
    prev = f.theta.copy()
    worst = 0.0
    for b in range(len(ptr) - 1):
        theta = torch.tensor(f.theta, dtype=torch.float64, device="cuda")
        plan.sweep(theta, ptr[:b + 2], src[:ptr[b + 1]], 1, params)
        cur = theta.cpu().numpy()
        members = [int(s) for s in src[ptr[b]:ptr[b + 1]]]
        others = np.ones(f.n_src, bool)
        others[members] = False
        np.testing.assert_array_equal(cur[others], prev[others])
        for s in members:
            bound, row, _, _ = newton_step_bound(N, f, prev, s, params.radius0)
            diff = np.abs(cur[s, :len(row)] - row)
            assert np.all(diff <= bound), (b, s, (diff / np.maximum(bound, 1e-300)).max())
            worst = max(worst, float(np.max(np.where(bound > 0, diff / np.maximum(bound, 1e-300), 0.0))))
        say("  batch", b, "members", members, "worst |diff| / bound %.3g" % worst)
        prev = cur
    return prev, worst
