"""Pins of the FP64 oracle against closed forms, library routines, Monte Carlo and
invariants.  None of these re-type the oracle's formulas: each checks a fact that the
model's definition fixes independently of how the oracle writes it.

Model reference: Regier et al. 2018, Section III (Poisson pixels, latent type,
log-normal reference-band brightness, Gaussian colours) and Eq. (1) (the ELBO).
"""
import numpy as np
import pytest
from scipy import stats
from scipy.special import gammaln

from conftest import clone, single_source

B = np.array([[-1, -1, 0, 0], [0, -1, 0, 0], [0, 0, 0, 0], [0, 0, 1, 0], [0, 0, 1, 1]])


def rotation(phi):
    return np.array([[np.cos(phi), -np.sin(phi)], [np.sin(phi), np.cos(phi)]])


def shape_cov(rho, phi, re):
    R = rotation(phi)
    return re ** 2 * R @ np.diag([1.0, rho ** 2]) @ R.T


def scipy_profiles(f, s, n, pts):
    """Star and galaxy profiles from scipy's multivariate normal (world position and shape
    mapped to the image frame by the image's linear astrometry)."""
    th = f.theta[s]
    A = f.wcs(n)
    u = A @ (th[:2] - f.img_origin[n])
    Ss = A @ shape_cov(th[3], th[4], th[5]) @ A.T
    fs = np.zeros(len(pts))
    fd = np.zeros(len(pts))
    fe = np.zeros(len(pts))
    for k in range(3):
        w, xi, Sk = f.img_psf[n, k, 0], f.img_psf[n, k, 1:3], f.img_psf[n, k, [3, 4, 4, 5]].reshape(2, 2)
        fs += w * stats.multivariate_normal(u + xi, Sk).pdf(pts)
        for a, nu in zip(f.dev_alpha, f.dev_nu):
            fd += w * a * stats.multivariate_normal(u + xi, nu * Ss + Sk).pdf(pts)
        for a, nu in zip(f.exp_alpha, f.exp_nu):
            fe += w * a * stats.multivariate_normal(u + xi, nu * Ss + Sk).pdf(pts)
    return fs, th[2] * fd + (1 - th[2]) * fe


# ------------------------------------------------------------------ P1: Gaussians
def test_p1_profiles_match_scipy(synth, O):
    f = synth.tiny(S=1, n_bands=2, size=21, side=21, seed=11, psf_xi=True, anisotropic_psf=True)
    f.theta[0, 2:6] = [0.3, 0.45, 0.7, 2.2]
    f.img_origin[1] = [0.25, -0.5]
    P = O.Problem(f)
    rng = np.random.default_rng(0)
    pts = rng.uniform(0, 20, (40, 2))
    for n in range(2):
        fs, fg = scipy_profiles(f, 0, n, pts)
        got = np.array([O.profiles(P, 0, n, p[0], p[1]) for p in pts])
        np.testing.assert_allclose(got[:, 0], fs, rtol=1e-12, atol=0)
        np.testing.assert_allclose(got[:, 1], fg, rtol=1e-12, atol=0)


def test_p1_galaxy_second_moments_fix_axis_conventions(synth, O):
    """Light of a galaxy: second central moments = sum_j alpha_j nu_j Sigma_s + PSF; the
    major axis (eigenvalue radius^2) points along angle phi, the minor one has
    (ratio * radius)^2."""
    size = 181
    rho, phi, re = 0.4, 0.6, 6.0
    f = single_source(synth, size=size, shape=[0.0, rho, phi, re], psf_sigmas=[1.2, 1.2, 1.2],
                      q=0.5)
    P = O.Problem(f)
    # galaxy only: q -> tiny so the star part vanishes from E_s
    f.theta[0, 6] = 1e-12
    P = O.Problem(f)
    E, _ = O.source_light(P, f, 0, 0)
    yy, xx = np.mgrid[0:size, 0:size].astype(float)
    m = E.sum()
    cx, cy = (E * xx).sum() / m, (E * yy).sum() / m
    np.testing.assert_allclose([cx, cy], f.theta[0, :2], atol=1e-6)
    M = np.array([[(E * (xx - cx) ** 2).sum(), (E * (xx - cx) * (yy - cy)).sum()],
                  [(E * (xx - cx) * (yy - cy)).sum(), (E * (yy - cy) ** 2).sum()]]) / m
    gal = (M - 1.2 ** 2 * np.eye(2)) / np.sum(f.exp_alpha * f.exp_nu)
    evals, evecs = np.linalg.eigh(gal)
    np.testing.assert_allclose(evals, [(rho * re) ** 2, re ** 2], rtol=2e-3)
    major = evecs[:, 1]
    assert abs(abs(major @ [np.cos(phi), np.sin(phi)]) - 1.0) < 1e-4


# ------------------------------------------------------------------ P2: brightness
def test_p2_flux_moments_monte_carlo(synth, O):
    f = synth.tiny(S=1, n_bands=1, seed=2)
    f.theta[0, 7:17] = [6.5, 0.2, 0.3, -0.4, 0.5, -0.2, 0.05, 0.1, 0.15, 0.08]
    f.theta[0, 17:27] = [7.0, 0.1, -0.3, 0.2, 0.1, 0.4, 0.12, 0.03, 0.07, 0.2]
    P = O.Problem(f)
    rng = np.random.default_rng(1)
    N = 1_000_000
    for a, base in ((0, 7), (1, 17)):
        th = f.theta[0, base:base + 10]
        logr = rng.normal(th[0], np.sqrt(th[1]), N)
        col = rng.normal(th[2:6], np.sqrt(th[6:10]), (N, 4))
        fl = synth._band_fluxes(np.exp(logr), col)   # definition of colours, from the generator
        for b in range(5):
            m1, m2 = O.flux_moments(P, 0, a, b)
            x = fl[:, b]
            se1 = x.std() / np.sqrt(N)
            se2 = (x ** 2).std() / np.sqrt(N)
            assert abs(x.mean() - m1) < 4 * se1, (a, b, x.mean(), m1)
            assert abs((x ** 2).mean() - m2) < 4 * se2, (a, b)


# ------------------------------------------------------------------ P3: E[F], Var[F]
def test_p3_pixel_moments_monte_carlo(synth, O):
    f = synth.tiny(S=3, n_bands=1, size=7, side=7, seed=5)
    f.img_band[:] = 1
    f.img_iota[:] = 1.7
    for s in range(3):
        f.theta[s, 8] = 0.25
        f.theta[s, 18] = 0.15
        f.theta[s, 13:17] = 0.05
        f.theta[s, 23:27] = 0.08
    f.theta[:, 6] = [0.3, 0.6, 0.85]
    f.boxes[:, 1:] = [0, 0, 7, 7]          # every source covers every pixel
    P = O.Problem(f)
    E, V = O.render(P, f, 0)
    yy, xx = np.mgrid[0:7, 0:7]
    pts = np.stack([xx.ravel(), yy.ravel()], 1).astype(float)
    profs = [scipy_profiles(f, s, 0, pts) for s in range(3)]
    rng = np.random.default_rng(2)
    N, chunk = 1_000_000, 100_000
    s1 = np.zeros(49)
    s2 = np.zeros(49)
    s4 = np.zeros(49)
    samples = []
    for _ in range(N // chunk):
        F = np.full((chunk, 49), f.img_sky[0])
        for s in range(3):
            th = f.theta[s]
            star = rng.random(chunk) < th[6]
            for a, base, prof in ((0, 7, profs[s][0]), (1, 17, profs[s][1])):
                logr = rng.normal(th[base], np.sqrt(th[base + 1]), chunk)
                col = rng.normal(th[base + 2:base + 6], np.sqrt(th[base + 6:base + 10]), (chunk, 4))
                fl = synth._band_fluxes(np.exp(logr), col)[:, 1]
                sel = star if a == 0 else ~star
                F[sel] += f.img_iota[0] * fl[sel, None] * prof[None, :]
        samples.append(F)
        s1 += F.sum(0)
    mean = s1 / N
    for F in samples:
        d = F - mean
        s2 += (d ** 2).sum(0)
        s4 += (d ** 4).sum(0)
    var = s2 / (N - 1)
    se_mean = np.sqrt(var / N)
    se_var = np.sqrt((s4 / N - var ** 2) / N)
    assert np.all(np.abs(mean - E.ravel()) < 4.5 * se_mean)
    assert np.all(np.abs(var - V.ravel()) < 4.5 * se_var)


# ------------------------------------------------------------------ P4/P5: delta method
@pytest.mark.parametrize("is_star", [True, False])
def test_p5_zero_variance_is_poisson_loglik(synth, O, is_star):
    """With (numerically) zero brightness variances and a known type, the ELBO's pixel
    part is the Poisson log-likelihood at the mean rate (with the log x! constant)."""
    f = single_source(synth, size=15, shape=[0.35, 0.6, 1.1, 1.8], q=1.0 if is_star else 0.0,
                      r_var=1e-30, c_var=1e-30, n_bands=2, band0=1, sky=120.0)
    f.flags = synth.FLAG_INCLUDE_LGAMMA
    P = O.Problem(f)
    yy, xx = np.mgrid[0:15, 0:15]
    pts = np.stack([xx.ravel(), yy.ravel()], 1).astype(float)
    total = 0.0
    base = 7 if is_star else 17
    th = f.theta[0]
    for n in range(2):
        b = int(f.img_band[n])
        logflux = th[base] + B[b] @ th[base + 2:base + 6]
        fs, fg = scipy_profiles(f, 0, n, pts)
        lam = f.img_sky[n] + f.img_iota[n] * np.exp(logflux) * (fs if is_star else fg)
        total += stats.poisson.logpmf(f.image(n).ravel(), lam).sum()
    got = O.source_value(P, 0)
    np.testing.assert_allclose(got[0], total, rtol=1e-12)


def test_p4_delta_method_gap_is_second_order(synth, O):
    """One star, sky 0, r band: E[log F] is exactly log iota + r_mu + log f, so the ELBO
    pixel part minus its exact counterpart is the delta-method error, which must scale
    as -(sum x) v^2 / 4 to leading order in the log-variance v."""
    gaps = []
    vs = [0.04, 0.02, 0.01]
    for v in vs:
        f = single_source(synth, size=11, q=1.0, r_var=v, c_var=0.0, sky=0.0, n_bands=1, band0=2,
                          psf_sigmas=[1.5, 2.0, 2.5])
        f.flags = 0
        P = O.Problem(f)
        yy, xx = np.mgrid[0:11, 0:11]
        pts = np.stack([xx.ravel(), yy.ravel()], 1).astype(float)
        fs, _ = scipy_profiles(f, 0, 0, pts)
        x = f.image(0).ravel()
        th = f.theta[0]
        iota = f.img_iota[0]
        exact = np.sum(x * (np.log(iota) + th[7] + np.log(fs)) - iota * np.exp(th[7] + v / 2) * fs)
        gaps.append(O.source_value(P, 0)[0] - exact)
        sx = x.sum()
        ratio = gaps[-1] / (-sx * v ** 2 / 4)
        assert 1.0 <= ratio <= 1.0 + v, (v, ratio)


# ------------------------------------------------------------------ P6/P7: mass and tables
def test_p6_mixture_mass(synth, O):
    f = single_source(synth, size=121, shape=[0.6, 0.5, 0.3, 1.5], q=0.35,
                      psf_sigmas=[1.0, 1.7, 2.6], n_bands=3, band0=0)
    P = O.Problem(f)
    for n in range(3):
        E, _ = O.source_light(P, f, 0, n)
        b = int(f.img_band[n])
        m1s, _ = O.flux_moments(P, 0, 0, b)
        m1g, _ = O.flux_moments(P, 0, 1, b)
        q = f.theta[0, 6]
        expect = f.img_iota[n] * (q * m1s + (1 - q) * m1g)
        np.testing.assert_allclose(E.sum(), expect, rtol=1e-6)


@pytest.mark.parametrize("kind", ["exp", "dev"])
def test_p7_profile_tables(synth, kind):
    ea, en, da, dn, _, _ = synth.load_profiles()
    a, nu = (ea, en) if kind == "exp" else (da, dn)
    assert len(a) == (6 if kind == "exp" else 8)
    np.testing.assert_allclose(a.sum(), 1.0, atol=1e-14)
    # fraction of light inside radius 1 of an isotropic 2-D Gaussian of variance nu is
    # 1 - exp(-1/(2 nu)) (Rayleigh radius); the mixture's must be one half
    np.testing.assert_allclose(np.sum(a * (1 - np.exp(-1 / (2 * nu)))), 0.5, atol=1e-12)
    rng = np.random.default_rng(3)
    N = 2_000_000
    j = rng.choice(len(a), size=N, p=a)
    r = np.hypot(*rng.normal(0, 1, (2, N))) * np.sqrt(nu[j])
    frac = np.mean(r < 1.0)
    assert abs(frac - 0.5) < 4 * np.sqrt(0.25 / N)


# ------------------------------------------------------------------ P8: symmetries
def _elbo_grad(O, f):
    P = O.Problem(f)
    val, g, ga = O.source_grad(P, 0)
    return val[0] + val[1], g, ga


def test_p8_angle_period_and_round_galaxy(synth, O):
    f = single_source(synth, size=21, shape=[0.4, 0.55, 0.8, 2.0], q=0.4, n_bands=2)
    e0, g0, _ = _elbo_grad(O, f)
    f2 = clone(f)
    f2.theta[0, 4] += np.pi
    e1, g1, _ = _elbo_grad(O, f2)
    np.testing.assert_allclose(e1, e0, rtol=1e-14)
    np.testing.assert_allclose(g1, g0, rtol=1e-9, atol=1e-9 * np.abs(g0).max())
    f3 = clone(f)
    f3.theta[0, 3] = 1.0
    _, g3, ga3 = _elbo_grad(O, f3)
    assert abs(g3[4]) <= 1e-12 * ga3[4]


def _rot90(f, N):
    """Rotate a square one-source problem by +90 degrees: (x, y) -> (N-1-y, x)."""
    g = clone(f)
    for n in range(f.n_img):
        im = f.image(n)
        new = np.empty_like(im)
        for r in range(N):
            for c in range(N):
                # old pixel (x=c, y=r) lands at (x'=N-1-r, y'=c)
                new[c, N - 1 - r] = im[r, c]
        o = int(f.img_off[n])
        g.x[o:o + N * N] = new.ravel()
    ux, uy = f.theta[0, 0], f.theta[0, 1]
    g.theta[0, 0], g.theta[0, 1] = N - 1 - uy, ux
    g.theta[0, 4] = f.theta[0, 4] + np.pi / 2
    b = f.boxes.copy()
    g.boxes[:, 1] = b[:, 2]
    g.boxes[:, 2] = N - b[:, 1] - b[:, 3]
    g.boxes[:, 3] = b[:, 4]
    g.boxes[:, 4] = b[:, 3]
    return g


def test_p8_rotation_by_90_degrees(synth, O):
    N = 19
    f = single_source(synth, size=N, side=15, shape=[0.4, 0.5, 0.3, 2.2], q=0.45, n_bands=2,
                      center=8.7)
    f.theta[0, 1] = 9.2
    e0, g0, _ = _elbo_grad(O, f)
    e1, g1, _ = _elbo_grad(O, _rot90(f, N))
    np.testing.assert_allclose(e1, e0, rtol=1e-13)
    # d/dux = d/duy' ; d/duy = -d/dux'
    np.testing.assert_allclose([g0[0], g0[1]], [g1[1], -g1[0]], rtol=1e-8)
    np.testing.assert_allclose(g0[2:], g1[2:], rtol=1e-8, atol=1e-9 * np.abs(g0).max())


def test_p8_reflection(synth, O):
    N = 19
    f = single_source(synth, size=N, side=15, shape=[0.7, 0.35, 0.5, 1.7], q=0.5, n_bands=1,
                      center=9.3)
    e0, g0, _ = _elbo_grad(O, f)
    g = clone(f)
    g.x[:N * N] = f.image(0)[:, ::-1].ravel()
    g.theta[0, 0] = N - 1 - f.theta[0, 0]
    g.theta[0, 4] = -f.theta[0, 4]
    g.boxes[:, 2] = N - f.boxes[:, 2] - f.boxes[:, 4]
    e1, g1, _ = _elbo_grad(O, g)
    np.testing.assert_allclose(e1, e0, rtol=1e-13)
    np.testing.assert_allclose(g1[0], -g0[0], rtol=1e-8)
    np.testing.assert_allclose(g1[4], -g0[4], rtol=1e-8)
    np.testing.assert_allclose(g1[5:], g0[5:], rtol=1e-8, atol=1e-9 * np.abs(g0).max())


def test_p8_integer_translation(synth, O):
    N = 25
    f = single_source(synth, size=N, side=11, shape=[0.2, 0.7, 1.9, 1.4], q=0.6, center=9.4)
    e0, g0, _ = _elbo_grad(O, f)
    g = clone(f)
    im = f.image(0)
    sh = np.full_like(im, f.img_sky[0])
    sh[3:, 5:] = im[:-3, :-5]
    g.x[:N * N] = sh.ravel()
    g.theta[0, 0] += 5
    g.theta[0, 1] += 3
    g.boxes[:, 1] += 3
    g.boxes[:, 2] += 5
    e1, g1, _ = _elbo_grad(O, g)
    np.testing.assert_allclose(e1, e0, rtol=1e-13)
    np.testing.assert_allclose(g1, g0, rtol=1e-8, atol=1e-9 * np.abs(g0).max())


# ------------------------------------------------------------------ P9: linearity
def test_p9_linearity_in_iota_and_brightness(synth, O):
    f = synth.tiny(S=2, n_bands=2, size=13, side=13, seed=9)
    P = O.Problem(f)
    E0, V0 = O.render(P, f, 1)
    g = clone(f)
    g.img_iota[1] *= 2.0
    E1, V1 = O.render(O.Problem(g), g, 1)
    sky = f.img_sky[1]
    np.testing.assert_allclose(E1 - sky, 2 * (E0 - sky), rtol=1e-12)
    np.testing.assert_allclose(V1, 4 * V0, rtol=1e-12)
    h = clone(f)
    h.theta[0, 7] += np.log(2.0)
    h.theta[0, 17] += np.log(2.0)
    Ea, _ = O.source_light(P, f, 0, 0)
    Eb, _ = O.source_light(O.Problem(h), h, 0, 0)
    np.testing.assert_allclose(Eb, 2 * Ea, rtol=1e-12)


# ------------------------------------------------------------------ P10/P11: derivatives
def _fd_grad(O, f, s, h=1e-6):
    th = f.theta
    g = np.zeros(27)
    for i in range(27):
        step = h * max(1.0, abs(th[s, i]))
        tp, tm = th.copy(), th.copy()
        tp[s, i] += step
        tm[s, i] -= step
        g[i] = (O.source_elbo(O.Problem(f, tp), s) - O.source_elbo(O.Problem(f, tm), s)) / (2 * step)
    return g


def test_p10_gradient_vs_central_differences(synth, O):
    f = synth.tiny(S=3, n_bands=3, size=17, side=11, seed=21)
    for s in range(3):
        P = O.Problem(f)
        val, g, ga = O.source_grad(P, s)
        fd = _fd_grad(O, f, s)
        elbo = abs(val[0]) + abs(val[1])
        tol = 1e-5 * np.abs(g) + 50 * 2.2e-16 * elbo / 1e-6
        assert np.all(np.abs(fd - g) <= tol), (s, np.abs(fd - g) / tol)


def test_p11_hvp_vs_gradient_differences_and_symmetry(synth, O):
    f = synth.tiny(S=2, n_bands=2, size=15, side=11, seed=31)
    P = O.Problem(f)
    rng = np.random.default_rng(4)
    v = rng.standard_normal(27)
    w = rng.standard_normal(27)
    hv, ha = O.source_hvp(P, 0, v)
    hw, _ = O.source_hvp(P, 0, w)
    np.testing.assert_allclose(w @ hv, v @ hw, rtol=1e-10)
    scale = np.maximum(1.0, np.abs(f.theta[0, :27]))
    h = 1e-5
    tp, tm = f.theta.copy(), f.theta.copy()
    tp[0, :27] += h * v * scale
    tm[0, :27] -= h * v * scale
    gp = O.source_grad(O.Problem(f, tp), 0)[1]
    gm = O.source_grad(O.Problem(f, tm), 0)[1]
    fd = (gp - gm) / (2 * h)
    hv_scaled = O.source_hvp(P, 0, v * scale)[0]
    err = np.abs(fd - hv_scaled)
    assert np.all(err <= 1e-4 * np.abs(hv_scaled) + 1e-6 * np.abs(ha).max()), err


# ------------------------------------------------------------------ KL and P15
def test_kl_monte_carlo(synth, O):
    f = synth.tiny(S=1, n_bands=1, seed=12)
    f.theta[0, 6] = 0.3
    f.theta[0, 7:17] = [6.0, 0.3, 0.2, -0.1, 0.4, 0.0, 0.1, 0.2, 0.05, 0.3]
    f.theta[0, 17:27] = [7.5, 0.5, -0.2, 0.3, 0.1, -0.4, 0.2, 0.1, 0.15, 0.05]
    P = O.Problem(f)
    rng = np.random.default_rng(6)
    N = 2_000_000
    q = f.theta[0, 6]
    star = rng.random(N) < q
    lq = np.where(star, np.log(q), np.log(1 - q))
    lp = np.where(star, np.log(f.prior_phi), np.log(1 - f.prior_phi))
    for a, base in ((0, 7), (1, 17)):
        sel = star if a == 0 else ~star
        th = f.theta[0, base:base + 10]
        r = rng.normal(th[0], np.sqrt(th[1]), N)
        c = rng.normal(th[2:6], np.sqrt(th[6:10]), (N, 4))
        lq_a = stats.norm.logpdf(r, th[0], np.sqrt(th[1])) + \
            stats.norm.logpdf(c, th[2:6], np.sqrt(th[6:10])).sum(1)
        lp_a = stats.norm.logpdf(r, f.prior_r[a, 0], np.sqrt(f.prior_r[a, 1])) + \
            stats.norm.logpdf(c, f.prior_c[a, 0], np.sqrt(f.prior_c[a, 1])).sum(1)
        lq = lq + np.where(sel, lq_a, 0.0)
        lp = lp + np.where(sel, lp_a, 0.0)
    d = lq - lp
    assert abs(d.mean() - O.kl(P, 0)) < 4 * d.std() / np.sqrt(N)
    # KL vanishes when q equals the prior
    g = clone(f)
    g.theta[0, 6] = g.prior_phi
    for a, base in ((0, 7), (1, 17)):
        g.theta[0, base], g.theta[0, base + 1] = g.prior_r[a]
        g.theta[0, base + 2:base + 6] = g.prior_c[a, 0]
        g.theta[0, base + 6:base + 10] = g.prior_c[a, 1]
    assert abs(O.kl(O.Problem(g), 0)) < 1e-15


def test_p15_pixels_outside_own_boxes_do_not_matter(synth, O):
    f = synth.tiny(S=2, n_bands=2, size=21, side=7, seed=41)
    P = O.Problem(f)
    v0, g0, _ = O.source_grad(P, 0)
    g = clone(f)
    mask = np.ones(g.x.shape, bool)
    for b in range(g.patch_ptr[0], g.patch_ptr[1]):
        n, r0, c0, h, w = g.boxes[b]
        o = int(g.img_off[n])
        W = int(g.img_W[n])
        for r in range(r0, r0 + h):
            mask[o + r * W + c0:o + r * W + c0 + w] = False
    g.x[mask] += 7.0
    v1, g1, _ = O.source_grad(O.Problem(g), 0)
    np.testing.assert_array_equal(v1, v0)
    np.testing.assert_array_equal(g1, g0)


def test_total_elbo_equals_sum_when_boxes_disjoint(synth, O):
    f = synth.tiny(S=2, n_bands=2, size=31, side=7, seed=51)
    f.theta[0, :2] = [7.0, 7.0]
    f.theta[1, :2] = [22.0, 21.0]
    f.boxes[:, 1:3] = np.array([[4, 4], [4, 4], [18, 19], [18, 19]])
    P = O.Problem(f)
    tot = O.total_elbo(P)
    np.testing.assert_allclose(tot, O.source_elbo(P, 0) + O.source_elbo(P, 1), rtol=1e-14)


def _poisson_limit_field(synth, wcs=False):
    """Four sources with overlapping boxes of different sizes on two images, known types
    (q = 1 star, q = 0 galaxy) and numerically zero brightness and colour variances, so
    that every source's band flux is the deterministic exp(log flux)."""
    f = synth.tiny(S=4, n_bands=2, size=23, side=9, seed=97, psf_xi=True, anisotropic_psf=True, wcs=wcs)
    f.flags = synth.FLAG_INCLUDE_LGAMMA
    f.theta[:, 6] = [1.0, 0.0, 1.0, 0.0]
    f.theta[:, :2] = [[8.2, 8.9], [12.4, 11.1], [10.3, 14.6], [14.8, 9.7]]
    f.theta[:, 2:6] = [[0.2, 0.7, 0.4, 1.3], [0.6, 0.5, 1.9, 2.1], [0.9, 0.8, 2.5, 1.0],
                       [0.1, 0.3, 0.2, 1.7]]
    for base in (7, 17):
        f.theta[:, base + 1] = 1e-30
        f.theta[:, base + 6:base + 10] = 1e-30
    # boxes: (img, r0, c0, h, w); every pair of sources overlaps somewhere, some pixels are
    # covered by three or four boxes, and each box differs between the two images
    f.boxes = np.array([[0, 3, 2, 11, 13], [1, 4, 3, 9, 9],
                        [0, 5, 6, 13, 11], [1, 6, 7, 11, 9],
                        [0, 9, 4, 12, 12], [1, 8, 5, 13, 11],
                        [0, 2, 9, 15, 11], [1, 3, 10, 11, 10]], np.int32)
    f.patch_ptr = np.array([0, 2, 4, 6, 8], np.int32)
    return f


def _poisson_rates(f, n):
    """Sky plus the light of every source whose box in image n covers the pixel, at every
    pixel of image n (scipy densities); and the union of the boxes as a mask."""
    H, W = int(f.img_H[n]), int(f.img_W[n])
    yy, xx = np.mgrid[0:H, 0:W]
    pts = np.stack([xx.ravel(), yy.ravel()], 1).astype(float)
    lam = np.full(H * W, float(f.img_sky[n]))
    union = np.zeros((H, W), bool)
    b = int(f.img_band[n])
    for s in range(f.n_src):
        for img, r0, c0, h, w in f.boxes[f.patch_ptr[s]:f.patch_ptr[s + 1]]:
            if img != n:
                continue
            inbox = np.zeros((H, W), bool)
            inbox[r0:r0 + h, c0:c0 + w] = True
            union |= inbox
            th = f.theta[s]
            star = th[6] == 1.0
            base = 7 if star else 17
            flux = np.exp(th[base] + B[b] @ th[base + 2:base + 6])
            fs, fg = scipy_profiles(f, s, n, pts)
            lam += np.where(inbox.ravel(), f.img_iota[n] * flux * (fs if star else fg), 0.0)
    return lam, union.ravel()


@pytest.mark.parametrize("wcs", [False, True])
def test_total_elbo_overlapping_boxes_is_poisson_loglik_of_union(synth, O, wcs):
    """In the zero-variance, known-type limit the total ELBO is the Poisson log-likelihood
    of every pixel of the union of the boxes, each counted once, at the rate summed over the
    sources whose box covers it; a pixel counted twice, or a source added outside its box,
    fails.  Each source's ELBO_s is the same sum over its own boxes only."""
    f = _poisson_limit_field(synth, wcs=wcs)
    P = O.Problem(f)
    total = 0.0
    own = np.zeros(f.n_src)
    for n in range(f.n_img):
        lam, union = _poisson_rates(f, n)
        lp = stats.poisson.logpmf(f.image(n).ravel(), lam)
        total += lp[union].sum()
        H, W = int(f.img_H[n]), int(f.img_W[n])
        for s in range(f.n_src):
            for img, r0, c0, h, w in f.boxes[f.patch_ptr[s]:f.patch_ptr[s + 1]]:
                if img == n:
                    own[s] += lp.reshape(H, W)[r0:r0 + h, c0:c0 + w].sum()
    # the boxes really overlap: the union is smaller than the sum of the box areas
    assert sum(int(h * w) for _, _, _, h, w in f.boxes) > sum(
        int(_poisson_rates(f, n)[1].sum()) for n in range(f.n_img)) + 100
    np.testing.assert_allclose(O.total_elbo(P), total, rtol=1e-12)
    for s in range(f.n_src):
        np.testing.assert_allclose(O.source_value(P, s)[0], own[s], rtol=1e-12)


def test_masked_pixels_are_skipped(synth, O):
    f = synth.tiny(S=1, n_bands=1, size=11, side=11, seed=61)
    P = O.Problem(f)
    v0 = O.source_value(P, 0)
    _, r0, c0, h, w = f.boxes[0]
    k = (r0 + h // 2) * 11 + c0 + w // 2      # a pixel inside the source's box
    g = clone(f)
    g.x[k] = np.nan
    v1 = O.source_value(O.Problem(g), 0)
    h = clone(f)
    h.x[k] = 0.0
    # dropping the pixel equals the full sum minus that pixel's term; compare via the
    # difference of two unmasked evaluations differing only in x at that pixel
    v2 = O.source_value(O.Problem(h), 0)
    E, V = O.render(P, f, 0)
    term_x = v0[0] - v2[0]       # x * (log E - V / 2E^2) part for the original count
    np.testing.assert_allclose(v0[0] - v1[0], term_x - E.ravel()[k], rtol=1e-9)


def test_neighbourhood_reduction_keeps_source_terms(synth, O):
    """The test-side reduction to a source's overlapping neighbours leaves its ELBO and
    gradient unchanged (every pixel of its boxes sees the same sources)."""
    from conftest import neighbourhood
    f = synth.region_16src()
    P = O.Problem(f)
    for s in (0, 9):
        g, j = neighbourhood(f, s)
        assert 1 <= g.n_src <= f.n_src
        v_full, g_full, _ = O.source_grad(P, s)
        v_sub, g_sub, _ = O.source_grad(O.Problem(g), j)
        np.testing.assert_allclose(v_sub, v_full, rtol=1e-15, atol=0)
        np.testing.assert_allclose(g_sub, g_full, rtol=1e-14, atol=1e-14 * np.abs(g_full).max())


# ------------------------------------------------- image metadata: astrometry, sky maps
def test_wcs_profiles_match_scipy(synth, O):
    """With a rotated, scaled and sheared astrometry the profiles are the textbook densities
    at the mapped position with the mapped shape covariance."""
    f = synth.tiny(S=1, n_bands=2, size=21, side=21, seed=12, psf_xi=True, anisotropic_psf=True, wcs=True)
    f.theta[0, 2:6] = [0.35, 0.5, 0.9, 2.1]
    f.img_origin[1] = [0.4, -0.3]
    assert not np.allclose(f.wcs(1), np.eye(2))
    P = O.Problem(f)
    pts = np.random.default_rng(1).uniform(0, 20, (40, 2))
    for n in range(2):
        fs, fg = scipy_profiles(f, 0, n, pts)
        got = np.array([O.profiles(P, 0, n, p[0], p[1]) for p in pts])
        np.testing.assert_allclose(got[:, 0], fs, rtol=1e-12, atol=0)
        np.testing.assert_allclose(got[:, 1], fg, rtol=1e-12, atol=0)


def test_wcs_world_rotation_invariance(synth, O):
    """Rotating the world frame by R (position R u, angle phi + a, astrometry A R^T) leaves
    every pixel's rate unchanged: same ELBO, gradient in u rotated by R, the rest equal."""
    f = synth.tiny(S=2, n_bands=2, size=19, side=13, seed=13, wcs=True)
    f.theta[:, 2:6] = [[0.3, 0.6, 0.4, 1.8], [0.7, 0.4, 2.0, 1.3]]
    a = 0.7
    R = rotation(a)
    g = clone(f)
    g.img_wcs = np.stack([f.wcs(n) @ R.T for n in range(f.n_img)])
    g.img_origin = (R @ f.img_origin.T).T
    g.theta[:, :2] = (R @ f.theta[:, :2].T).T
    g.theta[:, 4] = f.theta[:, 4] + a
    P0, P1 = O.Problem(f), O.Problem(g)
    for s in range(2):
        v0, g0, _ = O.source_grad(P0, s)
        v1, g1, _ = O.source_grad(P1, s)
        np.testing.assert_allclose(v1[0] + v1[1], v0[0] + v0[1], rtol=1e-12)
        sc = np.abs(g0).max()
        np.testing.assert_allclose(g1[:2], R @ g0[:2], rtol=1e-8, atol=1e-10 * sc)
        np.testing.assert_allclose(g1[2:], g0[2:], rtol=1e-8, atol=1e-10 * sc)


def test_wcs_scale_equals_scaled_source(synth, O):
    """An astrometry s I is the identity astrometry with the source's offset from the origin
    and its radius scaled by s (the PSF lives in the image frame)."""
    f = synth.tiny(S=1, n_bands=1, size=23, side=23, seed=14)
    f.theta[0, :2] = [10.3, 11.6]
    f.theta[0, 2:6] = [0.4, 0.55, 1.1, 1.9]
    sc = 1.07
    g = clone(f)
    g.img_wcs = np.array([sc * np.eye(2)])
    h = clone(f)
    h.theta[0, :2] = sc * f.theta[0, :2]
    h.theta[0, 5] = sc * f.theta[0, 5]
    vg = O.source_value(O.Problem(g), 0)
    vh = O.source_value(O.Problem(h), 0)
    np.testing.assert_allclose(vg, vh, rtol=1e-12)


def test_sky_map_adds_per_pixel(synth, O):
    """E[F] over a sky map is the constant-sky E[F] plus (map - constant), pixel by pixel;
    a constant map or the identity astrometry changes no term at all."""
    f = synth.tiny(S=3, n_bands=2, size=17, side=11, seed=15, sky_map=True)
    assert f.sky_map is not None
    g = clone(f)
    g.sky_map = None
    P, Q = O.Problem(f), O.Problem(g)
    for n in range(2):
        E1, V1 = O.render(P, f, n)
        E0, V0 = O.render(Q, g, n)
        smap = f.sky_map[f.img_off[n]:f.img_off[n] + 17 * 17].reshape(17, 17)
        np.testing.assert_allclose(E1 - E0, smap - f.img_sky[n], rtol=0, atol=1e-12 * E0.max())
        np.testing.assert_array_equal(V1, V0)
    h = clone(g)
    h.sky_map = np.concatenate([np.full(17 * 17, g.img_sky[n]) for n in range(2)])
    h.img_wcs = np.stack([np.eye(2)] * 2)
    R = O.Problem(h)
    for s in range(3):
        np.testing.assert_array_equal(O.source_grad(R, s)[1], O.source_grad(Q, s)[1])


# ------------------------------------------------------------------ colour-prior mixture
def test_mixture_kl_monte_carlo(synth, O):
    """With the colour-prior mixture the KL is E_q[log q(a, r, c, z) - log p(a, r, c, z)]
    with the component indicator z ~ Cat(kappa) independent of the colours under q and
    p(c, z | a) = w_z N(c; mean_z, cov_z): Monte Carlo with 1e6 draws, scipy densities for
    the full-covariance prior components, within 4 standard errors."""
    f = synth.with_color_mixture(synth.tiny(S=1, n_bands=1, seed=41), seed=3)
    th = f.theta[0]
    th[6] = 0.35
    th[7:17] = [6.9, 0.3, 0.2, -0.3, 0.4, -0.1, 0.05, 0.2, 0.1, 0.12]
    th[17:27] = [7.2, 0.2, -0.4, 0.1, 0.3, 0.5, 0.15, 0.04, 0.09, 0.25]
    P = O.Problem(f)
    rng = np.random.default_rng(5)
    N = 1_000_000
    star = rng.random(N) < th[6]
    lq = np.where(star, np.log(th[6]), np.log1p(-th[6]))
    lp = np.where(star, np.log(f.prior_phi), np.log1p(-f.prior_phi))
    for t, base in ((0, 7), (1, 17)):
        m = star if t == 0 else ~star
        n = int(m.sum())
        r = rng.normal(th[base], np.sqrt(th[base + 1]), n)
        c = rng.normal(th[base + 2:base + 6], np.sqrt(th[base + 6:base + 10]), (n, 4))
        kap = th[27 + 8 * t:35 + 8 * t]
        z = rng.choice(8, size=n, p=kap / kap.sum())
        lqt = (stats.norm.logpdf(r, th[base], np.sqrt(th[base + 1]))
               + stats.norm.logpdf(c, th[base + 2:base + 6], np.sqrt(th[base + 6:base + 10])).sum(1)
               + np.log(kap[z]))
        lpt = stats.norm.logpdf(r, f.prior_r[t, 0], np.sqrt(f.prior_r[t, 1])) + np.log(f.color_mix_w[t][z])
        for d in range(8):
            sel = z == d
            lpt[sel] += stats.multivariate_normal(f.color_mix_mean[t, d], f.color_mix_cov[t, d]).logpdf(c[sel])
        lq[m] += lqt
        lp[m] += lpt
    d = lq - lp
    kl = O.kl(P, 0)
    assert abs(d.mean() - kl) < 4 * d.std() / np.sqrt(N), (d.mean(), kl, d.std() / np.sqrt(N))


def test_mixture_of_identical_components_reduces_to_single_prior(synth, O):
    """Eight identical components (weights 1/8, the single prior's mean and diagonal
    variances) with responsibilities 1/8: the categorical KL vanishes and the colour term
    is the single Gaussian prior's KL, so ELBO, KL and the gradient in the 27 shared
    parameters equal the oracle without the mixture."""
    f = synth.tiny(S=2, n_bands=2, size=15, side=9, seed=43)
    g = synth.with_color_mixture(f, seed=4, kappa="prior")
    g.color_mix_w = np.full((2, 8), 1.0 / 8)
    for t in range(2):
        g.color_mix_mean[t] = f.prior_c[t, 0]
        g.color_mix_cov[t] = np.diag(f.prior_c[t, 1])
    g.theta[:, 27:43] = 1.0 / 8
    P0, P1 = O.Problem(f), O.Problem(g)
    for s in range(2):
        np.testing.assert_allclose(O.kl(P1, s), O.kl(P0, s), rtol=1e-13)
        v0, g0, _ = O.source_grad(P0, s)
        v1, g1, _ = O.source_grad(P1, s)
        np.testing.assert_allclose(v1[:2], v0[:2], rtol=1e-13)
        np.testing.assert_allclose(g1[:27], g0, rtol=1e-12, atol=1e-12 * np.abs(g0).max())
        # d KL / d kappa_d = q_a (log(kappa_d / w_d) + 1 + KL_normal) is the same for every d
        for t, w in ((0, g.theta[s, 6]), (1, 1 - g.theta[s, 6])):
            kk = g1[27 + 8 * t:35 + 8 * t]
            np.testing.assert_allclose(kk, kk[0], rtol=1e-12)


def test_mixture_gradient_and_hvp_vs_finite_differences(synth, O):
    """The 43-direction dual-number gradient against central differences of the value
    (relative step 1e-6), and the Hessian-vector product against differences of the
    gradient, with the responsibilities moved off the simplex only infinitesimally (the
    oracle's KL is defined for any positive kappa)."""
    f = synth.with_color_mixture(synth.tiny(S=2, n_bands=2, size=13, side=9, seed=45), seed=5)
    P = O.Problem(f)
    s = 0
    _, g, _ = O.source_grad(P, s)
    assert g.shape == (43,)
    for i in list(range(0, 27, 3)) + list(range(27, 43)):
        h = 1e-6 * max(1.0, abs(f.theta[s, i]))
        tp, tm = f.theta.copy(), f.theta.copy()
        tp[s, i] += h
        tm[s, i] -= h
        fd = (O.source_elbo(O.Problem(f, tp), s) - O.source_elbo(O.Problem(f, tm), s)) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * abs(fd) + 1e-4, (i, g[i], fd)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(43)
    hv, _ = O.source_hvp(P, s, v)
    h = 1e-6
    tp, tm = f.theta.copy(), f.theta.copy()
    tp[s, :43] += h * v
    tm[s, :43] -= h * v
    fd = (O.source_grad(O.Problem(f, tp), s)[1] - O.source_grad(O.Problem(f, tm), s)[1]) / (2 * h)
    np.testing.assert_allclose(hv, fd, rtol=1e-5, atol=1e-4 * np.abs(fd).max())
    w = rng.standard_normal(43)
    hw, _ = O.source_hvp(P, s, w)
    np.testing.assert_allclose(w @ hv, v @ hw, rtol=1e-11)
