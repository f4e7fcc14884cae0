"""Seeded synthetic SDSS-shaped fields for the Celeste ELBO path.

This module only draws inputs: catalog truth, images, patch boxes and the starting
variational parameters.  It holds none of the ELBO's arithmetic (no mixture densities,
no moments, no likelihood): truth images are made by sampling photons, i.e. each
source emits Poisson(iota * flux) photons whose positions are drawn from its light
profile (an exact Sersic draw for galaxies) followed by a draw from the band's PSF,
and the photons are binned into pixels on top of Poisson sky counts.

Both the oracle tests and the GPU path take their inputs from here; nothing here
imports either of them.

Parameter layout of one source row theta[s, 0:48] (float64):
  0 u_x, 1 u_y        world position of the centre, pixels
  2 frac_dev          de Vaucouleurs fraction of the galaxy profile, [0, 1]
  3 axis_ratio        minor/major axis ratio, (0, 1]
  4 angle             major-axis angle counter-clockwise from +x, radians
  5 radius            half-light radius along the major axis, pixels (> 0)
  6 q_star            variational probability that the source is a star, (0, 1)
  7..16  star:   r_mu, r_var, c_mu[4], c_var[4]
  17..26 galaxy: r_mu, r_var, c_mu[4], c_var[4]
  27..34 star, 35..42 galaxy: responsibilities kappa[8] of the colour-prior mixture
         components (used with FLAG_COLOR_MIXTURE; zero otherwise)
  43..47 zero padding
r is the log reference-band (r-band) brightness, c_k = log(flux_{k+1} / flux_k) the
colours between adjacent bands u, g, r, i, z; the *_var entries are variances.
"""
from dataclasses import dataclass, field
import json
import os

import numpy as np

N_PARAM = 27
N_MIX = 8                  # components of each type's colour-prior mixture
N_PARAM_MIX = N_PARAM + 2 * N_MIX
I_KAPPA = 27
ROW = 48
I_UX, I_UY, I_FDEV, I_RHO, I_PHI, I_RE, I_Q = range(7)
I_STAR = 7
I_GAL = 17
N_BANDS = 5
REF_BAND = 2
FLAG_INCLUDE_KL = 1
FLAG_INCLUDE_LGAMMA = 2
FLAG_COLOR_MIXTURE = 4

_PROFILE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "profiles.json")


def load_profiles():
    with open(_PROFILE_PATH) as f:
        d = json.load(f)
    return (np.array(d["exp"]["alpha"]), np.array(d["exp"]["nu"]),
            np.array(d["dev"]["alpha"]), np.array(d["dev"]["nu"]),
            d["exp"]["b_n"], d["dev"]["b_n"])


@dataclass
class Field:
    """A problem: images, per-source patch boxes, starting theta and model constants."""
    img_band: np.ndarray        # int32 [n_img]
    img_H: np.ndarray           # int32 [n_img]
    img_W: np.ndarray           # int32 [n_img]
    img_off: np.ndarray         # int64 [n_img]  offset of image n in x
    img_sky: np.ndarray         # f64 [n_img]    sky level epsilon_n, e- per pixel
    img_iota: np.ndarray        # f64 [n_img]    calibration iota_n
    img_origin: np.ndarray      # f64 [n_img, 2] world (x, y) of pixel (row 0, col 0)
    img_psf: np.ndarray         # f64 [n_img, 3, 6] (w, xi_x, xi_y, S_xx, S_xy, S_yy)
    x: np.ndarray               # f64 [n_pix] pixel counts, row-major per image
    patch_ptr: np.ndarray       # int32 [S + 1]
    boxes: np.ndarray           # int32 [n_box, 5] (img, r0, c0, h, w)
    theta: np.ndarray           # f64 [S, 48]
    exp_alpha: np.ndarray
    exp_nu: np.ndarray
    dev_alpha: np.ndarray
    dev_nu: np.ndarray
    prior_phi: float            # prior probability of a star
    prior_r: np.ndarray         # f64 [2, 2]    (type, mean/var) of log r-band brightness
    prior_c: np.ndarray         # f64 [2, 2, 4] (type, mean/var, colour k)
    flags: int = FLAG_INCLUDE_KL
    truth: dict = field(default_factory=dict)
    name: str = ""
    img_wcs: np.ndarray = None  # f64 [n_img, 2, 2] image offset = wcs @ world offset; None: identity
    sky_map: np.ndarray = None  # f64 [n_pix] per-pixel sky level, layout of x; None: img_sky
    # colour prior as a Gaussian mixture per type (with FLAG_COLOR_MIXTURE)
    color_mix_w: np.ndarray = None      # f64 [2, 8] component weights (sum 1)
    color_mix_mean: np.ndarray = None   # f64 [2, 8, 4]
    color_mix_cov: np.ndarray = None    # f64 [2, 8, 4, 4] symmetric positive definite

    def wcs(self, n):
        return np.eye(2) if self.img_wcs is None else np.asarray(self.img_wcs[n], np.float64)

    @property
    def n_src(self):
        return int(self.theta.shape[0])

    @property
    def n_img(self):
        return int(self.img_band.shape[0])

    def image(self, n):
        o = int(self.img_off[n])
        return self.x[o:o + int(self.img_H[n]) * int(self.img_W[n])].reshape(
            int(self.img_H[n]), int(self.img_W[n]))

    def visits(self):
        b = self.boxes
        return int(np.sum(b[:, 3].astype(np.int64) * b[:, 4].astype(np.int64)))


# ----------------------------------------------------------------------------------
# drawing helpers


def _workers():
    env = os.environ.get("SYNTH_WORKERS") or os.environ.get("OMP_NUM_THREADS")
    n = int(env) if env else (os.cpu_count() or 1)
    return max(1, min(n, 16))


def _psf_draw(rng, n_img):
    """Per image: 3-component isotropic PSF, weights Dirichlet(5,3,2), sigma U[1,3] px."""
    psf = np.zeros((n_img, 3, 6))
    for n in range(n_img):
        w = rng.dirichlet([5.0, 3.0, 2.0])
        sig = rng.uniform(1.0, 3.0, size=3)
        psf[n, :, 0] = w
        psf[n, :, 3] = sig ** 2
        psf[n, :, 5] = sig ** 2
    return psf


def _band_fluxes(ref_flux, colours):
    """Fluxes in u..z from the r-band flux and the 4 adjacent-band log ratios."""
    f = np.zeros(colours.shape[:-1] + (N_BANDS,))
    f[..., REF_BAND] = ref_flux
    f[..., 3] = f[..., 2] * np.exp(colours[..., 2])
    f[..., 4] = f[..., 3] * np.exp(colours[..., 3])
    f[..., 1] = f[..., 2] * np.exp(-colours[..., 1])
    f[..., 0] = f[..., 1] * np.exp(-colours[..., 0])
    return f


def _sample_offsets(rng, kind, fdev, rho, phi, re, b_exp, b_dev):
    """Photon offsets from the source centre, before the PSF.

    kind 0 = point source; kind 1 = galaxy: with prob fdev a Sersic-4 draw, else Sersic-1.
    A Sersic-n radius (in half-light units) is (t / b_n)^n with t ~ Gamma(2n); the draw is
    scaled by radius along the major axis and radius*rho along the minor axis, then rotated.
    """
    n = kind.shape[0]
    dx = np.zeros(n)
    dy = np.zeros(n)
    g = kind == 1
    ng = int(g.sum())
    if ng:
        is_dev = rng.random(ng) < fdev[g]
        shape = np.where(is_dev, 8.0, 2.0)
        bn = np.where(is_dev, b_dev, b_exp)
        nn = np.where(is_dev, 4.0, 1.0)
        t = rng.gamma(shape)
        r = (t / bn) ** nn
        ang = rng.uniform(0.0, 2.0 * np.pi, ng)
        xm = re[g] * r * np.cos(ang)
        ym = re[g] * rho[g] * r * np.sin(ang)
        c, s = np.cos(phi[g]), np.sin(phi[g])
        dx[g] = c * xm - s * ym
        dy[g] = s * xm + c * ym
    return dx, dy


def _render_image(rng, H, W, sky, iota, origin, psf, band, src_pos, src_kind, src_flux,
                  src_shape, b_exp, b_dev, max_photons_chunk=1_000_000, wcs=None, sky_map=None):
    """Poisson sky plus binned photons of every source (world positions src_pos).  A
    photon's world offset from its source maps to the image through wcs; the PSF blur is
    drawn in the image frame."""
    A = np.eye(2) if wcs is None else np.asarray(wcs, np.float64)
    img = rng.poisson(sky if sky_map is None else sky_map, size=(H, W)).astype(np.float64)
    lam = iota * src_flux[:, band]
    # only sources whose light can reach the image (generous 300 px margin)
    wx = src_pos[:, 0] - origin[0]
    wy = src_pos[:, 1] - origin[1]
    px = A[0, 0] * wx + A[0, 1] * wy
    py = A[1, 0] * wx + A[1, 1] * wy
    near = (px > -300) & (px < W + 300) & (py > -300) & (py < H + 300)
    idx = np.nonzero(near)[0]
    if idx.size == 0:
        return img
    counts = rng.poisson(lam[idx])
    # process in chunks of sources to bound memory; bin once at the end
    hits = []
    start = 0
    while start < idx.size:
        stop = start
        tot = 0
        while stop < idx.size and (tot + counts[stop] <= max_photons_chunk or stop == start):
            tot += counts[stop]
            stop += 1
        sel = idx[start:stop]
        cnt = counts[start:stop]
        rep = np.repeat(np.arange(sel.size), cnt)
        if rep.size:
            s = sel[rep]
            fdev, rho, phi, re = (src_shape[s, 0], src_shape[s, 1], src_shape[s, 2],
                                  src_shape[s, 3])
            dx, dy = _sample_offsets(rng, src_kind[s], fdev, rho, phi, re, b_exp, b_dev)
            cw = np.cumsum(psf[:, 0]) / psf[:, 0].sum()
            k = np.minimum(np.searchsorted(cw, rng.random(rep.size), side="right"), 2)
            sig = np.sqrt(psf[k, 3])
            ex = psf[k, 1] + sig * rng.standard_normal(rep.size)
            ey = psf[k, 2] + sig * rng.standard_normal(rep.size)
            xx = px[s] + A[0, 0] * dx + A[0, 1] * dy + ex
            yy = py[s] + A[1, 0] * dx + A[1, 1] * dy + ey
            col = np.floor(xx + 0.5).astype(np.int64)
            row = np.floor(yy + 0.5).astype(np.int64)
            ok = (col >= 0) & (col < W) & (row >= 0) & (row < H)
            hits.append((row[ok] * W + col[ok]).astype(np.int32))
        start = stop
    if hits:
        img += np.bincount(np.concatenate(hits), minlength=H * W).reshape(H, W)
    return img


def _box(center_img, side_h, side_w, H, W):
    """Odd-sided box centred on the pixel nearest the centre, clipped to the image."""
    cx = int(np.floor(center_img[0] + 0.5))
    cy = int(np.floor(center_img[1] + 0.5))
    hh, hw = side_h // 2, side_w // 2
    r0, r1 = max(cy - hh, 0), min(cy + hh + 1, H)
    c0, c1 = max(cx - hw, 0), min(cx + hw + 1, W)
    if r1 <= r0 or c1 <= c0:
        return None
    return (r0, c0, r1 - r0, c1 - c0)


def _theta_from_truth(rng, pos, ref_flux, colours, shape, q_range=(0.1, 0.9), pos_sd=0.5):
    """Starting variational parameters: truth plus perturbation (sigma 0.1 on log scales)."""
    S = pos.shape[0]
    th = np.zeros((S, ROW))
    th[:, I_UX] = pos[:, 0] + rng.normal(0.0, pos_sd, S)
    th[:, I_UY] = pos[:, 1] + rng.normal(0.0, pos_sd, S)
    th[:, I_FDEV] = shape[:, 0]
    th[:, I_RHO] = shape[:, 1]
    th[:, I_PHI] = shape[:, 2]
    th[:, I_RE] = shape[:, 3]
    th[:, I_Q] = rng.uniform(q_range[0], q_range[1], S)
    for base in (I_STAR, I_GAL):
        th[:, base] = np.log(ref_flux) + rng.normal(0.0, 0.1, S)
        th[:, base + 1] = 0.01
        th[:, base + 2:base + 6] = colours + rng.normal(0.0, 0.1, (S, 4))
        th[:, base + 6:base + 10] = 0.01
    return th


def _truth_draw(rng, S, star_prob, logr_mean, logr_sd, logr_range, re_range=(0.5, 5.0)):
    kind = (rng.random(S) >= star_prob).astype(np.int64)   # 0 star, 1 galaxy
    logr = rng.normal(logr_mean, logr_sd, S)
    if logr_range is not None:
        lo, hi = logr_range
        bad = (logr < lo) | (logr > hi)
        while bad.any():
            logr[bad] = rng.normal(logr_mean, logr_sd, int(bad.sum()))
            bad = (logr < lo) | (logr > hi)
    colours = rng.normal(0.0, 0.5, (S, 4))
    shape = np.stack([rng.uniform(0.0, 1.0, S), rng.uniform(0.2, 1.0, S),
                      rng.uniform(0.0, np.pi, S), rng.uniform(re_range[0], re_range[1], S)],
                     axis=1)
    return kind, np.exp(logr), colours, shape


def _priors(star_prob, logr_mean, logr_sd):
    prior_r = np.array([[logr_mean, logr_sd ** 2], [logr_mean, logr_sd ** 2]])
    prior_c = np.zeros((2, 2, 4))
    prior_c[:, 1, :] = 0.25
    return float(star_prob), prior_r, prior_c


def _assemble(rng, images_meta, pos, kind, flux, colours, shape, box_sides, theta,
              star_prob, logr_mean, logr_sd, name, render=True):
    ea, en, da, dn, b_exp, b_dev = load_profiles()
    n_img = len(images_meta)
    img_band = np.array([m["band"] for m in images_meta], np.int32)
    img_H = np.array([m["H"] for m in images_meta], np.int32)
    img_W = np.array([m["W"] for m in images_meta], np.int32)
    sizes = img_H.astype(np.int64) * img_W.astype(np.int64)
    img_off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    img_sky = np.array([m["sky"] for m in images_meta])
    img_iota = np.array([m.get("iota", 1.0) for m in images_meta])
    img_origin = np.array([m["origin"] for m in images_meta], np.float64).reshape(n_img, 2)
    img_psf = np.array([m["psf"] for m in images_meta])
    has_wcs = any("wcs" in m for m in images_meta)
    img_wcs = (np.array([m.get("wcs", np.eye(2)) for m in images_meta], np.float64).reshape(n_img, 2, 2)
               if has_wcs else None)
    sky_map = None
    if any("sky_map" in m for m in images_meta):
        sky_map = np.empty(int(sizes.sum()))
        for n, m in enumerate(images_meta):
            sm = m.get("sky_map")
            sky_map[img_off[n]:img_off[n] + sizes[n]] = (np.full(int(sizes[n]), img_sky[n]) if sm is None
                                                         else np.asarray(sm, np.float64).reshape(-1))
    band_flux = _band_fluxes(flux, colours)
    x = np.empty(int(sizes.sum()))
    # one independent stream per image (spawned from the field's stream), so images can
    # be drawn concurrently and the result does not depend on the number of workers
    streams = [np.random.default_rng(s) for s in
               np.random.SeedSequence(int(rng.integers(2 ** 63))).spawn(n_img)]

    def draw(n):
        r = streams[n]
        smap = None if sky_map is None else sky_map[img_off[n]:img_off[n] + sizes[n]].reshape(
            int(img_H[n]), int(img_W[n]))
        if render:
            im = _render_image(r, int(img_H[n]), int(img_W[n]), img_sky[n], img_iota[n],
                               img_origin[n], img_psf[n], int(img_band[n]), pos, kind,
                               band_flux, shape, b_exp, b_dev,
                               wcs=None if img_wcs is None else img_wcs[n], sky_map=smap)
        else:
            im = r.poisson(img_sky[n] if smap is None else smap,
                           size=(int(img_H[n]), int(img_W[n]))).astype(float)
        x[img_off[n]:img_off[n] + sizes[n]] = im.reshape(-1)

    workers = min(n_img, _workers())
    if workers > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(draw, range(n_img)))
    else:
        for n in range(n_img):
            draw(n)
    # patch boxes, centred on the starting position
    S = theta.shape[0]
    ptr = [0]
    boxes = []
    for s in range(S):
        for n in range(n_img):
            c = theta[s, :2] - img_origin[n]
            if img_wcs is not None:
                c = img_wcs[n] @ c
            b = _box(c, int(box_sides[s]), int(box_sides[s]), int(img_H[n]), int(img_W[n]))
            if b is not None:
                boxes.append((n,) + b)
        ptr.append(len(boxes))
    phi, prior_r, prior_c = _priors(star_prob, logr_mean, logr_sd)
    return Field(img_band=img_band, img_H=img_H, img_W=img_W, img_off=img_off,
                 img_sky=img_sky, img_iota=img_iota, img_origin=img_origin, img_psf=img_psf,
                 x=x, patch_ptr=np.array(ptr, np.int32),
                 boxes=np.array(boxes, np.int32).reshape(-1, 5), theta=theta,
                 exp_alpha=ea, exp_nu=en, dev_alpha=da, dev_nu=dn,
                 prior_phi=phi, prior_r=prior_r, prior_c=prior_c,
                 truth={"pos": pos, "kind": kind, "flux": flux, "colours": colours,
                        "shape": shape},
                 name=name, img_wcs=img_wcs, sky_map=sky_map)


def _realistic_meta(rng, meta, wcs=True, sky_map=True):
    """Adds per-image metadata beyond a constant sky and a pure translation: a local
    linear astrometry (rotation up to 0.3 rad, per-axis scale 0.97-1.03, small shear) and a
    smooth sky map (linear gradients up to +-20% and a 10% sinusoid around the level)."""
    for m in meta:
        if wcs:
            a = rng.uniform(-0.3, 0.3)
            R = np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])
            Sc = np.array([[rng.uniform(0.97, 1.03), rng.uniform(-0.02, 0.02)],
                           [0.0, rng.uniform(0.97, 1.03)]])
            m["wcs"] = Sc @ R
        if sky_map:
            H, W = m["H"], m["W"]
            rr, cc = np.meshgrid(np.arange(H) / max(H - 1, 1), np.arange(W) / max(W - 1, 1), indexing="ij")
            g = rng.uniform(-0.2, 0.2, 2)
            amp, f1, f2, ph = rng.uniform(0.0, 0.1), rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0), rng.uniform(0, 6.3)
            m["sky_map"] = m["sky"] * (1.0 + g[0] * (rr - 0.5) + g[1] * (cc - 0.5)
                                       + amp * np.sin(2 * np.pi * (f1 * rr + f2 * cc) + ph))
    return meta


def _single_field_images(rng, H, W, bands=range(N_BANDS), origin=(0.0, 0.0)):
    psf = _psf_draw(rng, len(list(bands)))
    return [{"band": b, "H": H, "W": W, "sky": float(rng.uniform(100.0, 500.0)),
             "origin": origin, "psf": psf[i]} for i, b in enumerate(bands)]


def _odd(side):
    return 2 * np.round((side - 1) / 2).astype(np.int64) + 1


# ----------------------------------------------------------------------------------
# the five workloads


def single_source(seed=None):
    """One source (star w.p. 0.5) centred in a 41x41 patch in each of 5 bands."""
    rng = np.random.default_rng(1000 if seed is None else seed)
    imgs = _single_field_images(rng, 41, 41)
    kind, flux, colours, shape = _truth_draw(rng, 1, 0.5, np.log(1000.0), 1.0, None)
    pos = np.array([[20.0, 20.0]])
    theta = _theta_from_truth(rng, pos, flux, colours, shape)
    return _assemble(rng, imgs, pos, kind, flux, colours, shape, np.array([41]), theta,
                     0.5, np.log(1000.0), 1.0, "single_source")


def region_16src(seed=None):
    """16 overlapping sources, uniform positions, 5-band 256x256 region, 61x61 patches."""
    rng = np.random.default_rng(1001 if seed is None else seed)
    imgs = _single_field_images(rng, 256, 256)
    S = 16
    kind, flux, colours, shape = _truth_draw(rng, S, 0.5, np.log(1000.0), 1.0, None)
    pos = rng.uniform(0.0, 255.0, (S, 2))
    theta = _theta_from_truth(rng, pos, flux, colours, shape)
    return _assemble(rng, imgs, pos, kind, flux, colours, shape, np.full(S, 61), theta,
                     0.5, np.log(1000.0), 1.0, "region_16src")


LOGR_MEAN_FIELD = 7.71
LOGR_SD_FIELD = 1.267
LOGR_RANGE_FIELD = (np.log(50.0), np.log(1e5))


def sdss_field(S=2000, H=1489, W=2048, seed=1002, render=True, name="field_2000src", realistic=False):
    """SDSS-shaped field: S sources uniform over a W x H frame (a Poisson process conditioned
    on its count), 40% stars, patch side log-uniform in [21, 101] px (odd), r-band
    brightness log-normal truncated to [50, 1e5] e-.  realistic=True adds a local linear
    astrometry and a sky map per image and sizes each patch by brightness and radius
    (odd side 10 log10(flux) + 4 radius + 5, clipped to [21, 101])."""
    rng = np.random.default_rng(seed)
    imgs = _single_field_images(rng, H, W)
    kind, flux, colours, shape = _truth_draw(rng, S, 0.4, LOGR_MEAN_FIELD, LOGR_SD_FIELD,
                                             LOGR_RANGE_FIELD)
    pos = np.stack([rng.uniform(0.0, W - 1.0, S), rng.uniform(0.0, H - 1.0, S)], axis=1)
    sides = _odd(np.exp(rng.uniform(np.log(21.0), np.log(101.0), S)))
    if realistic:
        _realistic_meta(np.random.default_rng(seed + 7919), imgs)
        sides = _odd(np.clip(10.0 * np.log10(flux) + 4.0 * shape[:, 3] + 5.0, 21.0, 101.0))
    theta = _theta_from_truth(rng, pos, flux, colours, shape)
    return _assemble(rng, imgs, pos, kind, flux, colours, shape, sides, theta,
                     0.4, LOGR_MEAN_FIELD, LOGR_SD_FIELD, name, render=render)


def field_2000src(seed=None, render=True):
    return sdss_field(2000, seed=1002 if seed is None else seed, render=render, name="field_2000src")


def field_1024src(seed=None, render=True):
    """1024 sources from the field generator, plus a seeded HVP direction per source."""
    f = sdss_field(1024, seed=1003 if seed is None else seed, render=render, name="field_1024src")
    rng = np.random.default_rng((1003 if seed is None else seed) + 77)
    v = np.zeros_like(f.theta)
    v[:, :N_PARAM] = rng.standard_normal((f.n_src, N_PARAM))
    f.truth["v"] = v
    return f


def sky_region(n_fx=4, n_fy=4, epochs=2, S=20000, H=1489, W=2048, overlap=128,
               max_offset=500.0, seed=1004, render=True, name="sky_region_20000src"):
    """n_fx x n_fy fields on a grid overlapping by `overlap` px, each seen in `epochs`
    epochs whose frames are shifted by U[0, max_offset)^2 px, with a PSF per
    (field, epoch, band); S sources uniform over the union of the grid."""
    rng = np.random.default_rng(seed)
    imgs = []
    for fy in range(n_fy):
        for fx in range(n_fx):
            for e in range(epochs):
                off = rng.uniform(0.0, max_offset, 2)
                origin = (fx * (W - overlap) + off[0], fy * (H - overlap) + off[1])
                imgs += _single_field_images(rng, H, W, origin=origin)
    span_x = (n_fx - 1) * (W - overlap) + W
    span_y = (n_fy - 1) * (H - overlap) + H
    kind, flux, colours, shape = _truth_draw(rng, S, 0.4, LOGR_MEAN_FIELD, LOGR_SD_FIELD,
                                             LOGR_RANGE_FIELD)
    pos = np.stack([rng.uniform(0.0, span_x, S), rng.uniform(0.0, span_y, S)], axis=1)
    sides = _odd(np.exp(rng.uniform(np.log(21.0), np.log(101.0), S)))
    theta = _theta_from_truth(rng, pos, flux, colours, shape)
    return _assemble(rng, imgs, pos, kind, flux, colours, shape, sides, theta,
                     0.4, LOGR_MEAN_FIELD, LOGR_SD_FIELD, name, render=render)


def sky_region_20000src(seed=None, render=True):
    return sky_region(seed=1004 if seed is None else seed, render=render)


def tiny(S=2, n_bands=2, size=15, side=9, seed=7, sky=(100.0, 200.0), psf_xi=False,
         anisotropic_psf=False, star_prob=0.5, wcs=False, sky_map=False):
    """Small problem for tests: S sources in a size x size region, one image per band."""
    rng = np.random.default_rng(seed)
    bands = list(range(n_bands)) if n_bands <= N_BANDS else list(range(N_BANDS))
    imgs = []
    for i, b in enumerate(bands):
        psf = _psf_draw(rng, 1)[0]
        if psf_xi:
            psf[:, 1:3] = rng.normal(0.0, 0.3, (3, 2))
        if anisotropic_psf:
            a = rng.uniform(1.0, 2.5, 3)
            c = rng.uniform(1.0, 2.5, 3)
            psf[:, 3] = a ** 2
            psf[:, 5] = c ** 2
            psf[:, 4] = rng.uniform(-0.4, 0.4, 3) * a * c
        imgs.append({"band": b, "H": size, "W": size,
                     "sky": float(rng.uniform(*sky)), "origin": (0.0, 0.0), "psf": psf})
    if wcs or sky_map:
        _realistic_meta(np.random.default_rng(seed + 7919), imgs, wcs=wcs, sky_map=sky_map)
    kind, flux, colours, shape = _truth_draw(rng, S, star_prob, np.log(1000.0), 1.0, None)
    pos = rng.uniform(size * 0.25, size * 0.75, (S, 2))
    theta = _theta_from_truth(rng, pos, flux, colours, shape)
    return _assemble(rng, imgs, pos, kind, flux, colours, shape, np.full(S, side), theta,
                     star_prob, np.log(1000.0), 1.0, "tiny")


def with_color_mixture(f, seed=0, kappa="random"):
    """A copy of field f whose colour prior is a Gaussian mixture of N_MIX components per
    type (seeded draws: Dirichlet(2) weights, N(0, 0.5^2) means, covariances B B^T / 8 +
    0.01 I with B standard normal), with FLAG_COLOR_MIXTURE set and the responsibilities
    kappa of every source drawn from Dirichlet(1) ("random") or set to the prior weights
    ("prior")."""
    import copy
    rng = np.random.default_rng(10_000 + seed)
    g = copy.copy(f)
    g.color_mix_w = rng.dirichlet(np.full(N_MIX, 2.0), 2)
    g.color_mix_mean = rng.normal(0.0, 0.5, (2, N_MIX, 4))
    Bm = rng.standard_normal((2, N_MIX, 4, 4))
    g.color_mix_cov = np.einsum("tdij,tdkj->tdik", Bm, Bm) / 8.0 + 0.01 * np.eye(4)
    th = np.array(f.theta, np.float64, copy=True)
    for t in range(2):
        cols = slice(I_KAPPA + N_MIX * t, I_KAPPA + N_MIX * (t + 1))
        if kappa == "prior":
            th[:, cols] = g.color_mix_w[t]
        else:
            th[:, cols] = rng.dirichlet(np.ones(N_MIX), th.shape[0])
    g.theta = th
    g.flags = int(f.flags) | FLAG_COLOR_MIXTURE
    return g

