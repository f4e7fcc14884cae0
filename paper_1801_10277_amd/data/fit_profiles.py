"""Fit the isotropic Gaussian-mixture approximations of the two galaxy light profiles.

The model renders a galaxy as a blend of an exponential disk (Sersic index 1) and a
de Vaucouleurs bulge (Sersic index 4), each approximated by a mixture of isotropic,
zero-mean 2-D Gaussians (6 for the exponential, 8 for de Vaucouleurs) so that
convolution with a Gaussian-mixture PSF stays closed-form.  The paper delegates the
profile model to the original Celeste model; the coefficient tables are not printed
there, so this script fits its own.

Profile (unit half-light radius):  I_n(r) ~ exp(-b_n r^(1/n)),  b_n solving
gamma(2n, b_n) = Gamma(2n)/2 (regularised lower incomplete gamma = 1/2).

Mixture:  M(r) = sum_j alpha_j / (2 pi nu_j) exp(-r^2 / (2 nu_j)).

Fit: least squares of (M - I_n) weighted by annulus area on r in (0, 8], in log-space
parameters.  Afterwards the table is normalised exactly:
  * sum_j alpha_j = 1 (unit total flux),
  * the half-light radius is exactly 1:  sum_j alpha_j (1 - exp(-1/(2 nu_j))) = 1/2,
    enforced by a common rescale of the nu_j (1-D root find).

Run:  python paper_1801_10277_amd/data/fit_profiles.py   (writes profiles.json beside it)
"""
import json
import os

import numpy as np
from scipy.optimize import brentq, least_squares
from scipy.special import gamma, gammaincinv


def sersic_b(n):
    return float(gammaincinv(2.0 * n, 0.5))


def sersic_norm(n, r):
    """Surface brightness of a unit-flux, unit half-light-radius Sersic profile."""
    b = sersic_b(n)
    total = 2.0 * np.pi * n * gamma(2.0 * n) / b ** (2.0 * n)
    return np.exp(-b * r ** (1.0 / n)) / total


def mixture(alpha, nu, r):
    return (alpha[None, :] / (2.0 * np.pi * nu[None, :]) *
            np.exp(-r[:, None] ** 2 / (2.0 * nu[None, :]))).sum(axis=1)


def half_light_residual(alpha, nu, scale):
    return float(np.sum(alpha * (1.0 - np.exp(-1.0 / (2.0 * nu * scale)))) - 0.5)


def fit(n, J, rmax=8.0):
    r = np.concatenate([np.geomspace(1e-4, 0.05, 200), np.linspace(0.05, rmax, 2000)[1:]])
    dr = np.gradient(r)
    w = np.sqrt(2.0 * np.pi * r * dr)
    target = sersic_norm(n, r)
    # initial variances log-spaced across the profile's scales
    lo, hi = (1e-3, 4.0) if n == 1 else (1e-6, 30.0)
    nu0 = np.geomspace(lo, hi, J)
    a0 = np.full(J, 1.0 / J)
    p0 = np.concatenate([np.log(a0), np.log(nu0)])

    def resid(p):
        a = np.exp(p[:J])
        nu = np.exp(p[J:])
        m = mixture(a, nu, r)
        return np.concatenate([w * (m - target),
                               [10.0 * (a.sum() - 1.0)],
                               [10.0 * half_light_residual(a, nu, 1.0)]])

    sol = least_squares(resid, p0, xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=20000)
    alpha = np.exp(sol.x[:J])
    nu = np.exp(sol.x[J:])
    order = np.argsort(nu)
    alpha, nu = alpha[order], nu[order]
    alpha = alpha / alpha.sum()
    scale = brentq(lambda s: half_light_residual(alpha, nu, s), 1e-3, 1e3, xtol=1e-15, rtol=1e-15)
    nu = nu * scale
    rms = float(np.sqrt(np.mean(((mixture(alpha, nu, r) - target) * w) ** 2)))
    return alpha, nu, rms


def main():
    out = {}
    for name, n, J in (("exp", 1, 6), ("dev", 4, 8)):
        alpha, nu, rms = fit(n, J)
        out[name] = {"sersic_n": n, "b_n": sersic_b(n),
                     "alpha": [float(v) for v in alpha], "nu": [float(v) for v in nu],
                     "fit_weighted_rms": rms}
        print(name, "alpha", alpha, "nu", nu, "rms", rms,
              "half-light check", half_light_residual(alpha, nu, 1.0))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
