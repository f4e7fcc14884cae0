"""The identity behind the closed-form Hessian's second-derivative pass: down a strip of
rows, z = P (m - mu) is affine in the row, so each weighted pixel sum of n times a polynomial
of degree <= 4 in z (the second derivatives of a Gaussian in position, frac_dev and shape)
equals a fixed combination of the strip's centred row moments U_m = sum_k t_k s_k^m.  This
test restates the per-pixel formulas and the moment expansion independently (numpy) and
checks them against each other on random components, strips and weights."""
import numpy as np
import pytest


def per_pixel(a, b, d, dx, dy, t, wt, sg, wnu, nu, L):
    j = dy + np.arange(L)
    zx, zy = a * dx + b * j, b * dx + d * j
    Dxx, Dxy, Dyy = zx * zx - a, zx * zy - b, zy * zy - d
    v = wnu * nu
    return {
        "XX": np.sum(t * wt * Dxx), "XY": np.sum(t * wt * Dxy), "YY": np.sum(t * wt * Dyy),
        "XF": np.sum(t * sg * zx), "YF": np.sum(t * sg * zy),
        "X_SXX": np.sum(t * wnu * zx * (Dxx - 2 * a)),
        "X_SXY": np.sum(t * wnu * (zx * (Dxy - b) - a * zy)),
        "X_SYY": np.sum(t * wnu * (zx * Dyy - 2 * b * zy)),
        "Y_SXX": np.sum(t * wnu * (zy * Dxx - 2 * b * zx)),
        "Y_SXY": np.sum(t * wnu * (zy * (Dxy - b) - d * zx)),
        "Y_SYY": np.sum(t * wnu * zy * (Dyy - 2 * d)),
        "F_SXX": np.sum(t * sg * nu * Dxx), "F_SXY": np.sum(t * sg * nu * Dxy),
        "F_SYY": np.sum(t * sg * nu * Dyy),
        # s_ij s_kl n = nu^2 n (D_ij D_kl - T_ij,kl) with the T of the closed-form derivation
        "SXX_SXX": np.sum(t * v * (Dxx * Dxx - (4 * a * Dxx + 2 * a * a))),
        "SXX_SXY": np.sum(t * v * (Dxx * Dxy - (2 * a * Dxy + 2 * b * Dxx + 2 * a * b))),
        "SXX_SYY": np.sum(t * v * (Dxx * Dyy - (4 * b * Dxy + 2 * b * b))),
        "SXY_SXY": np.sum(t * v * (Dxy * Dxy - (a * Dyy + 2 * b * Dxy + d * Dxx + a * d + b * b))),
        "SXY_SYY": np.sum(t * v * (Dxy * Dyy - (2 * b * Dyy + 2 * d * Dxy + 2 * b * d))),
        "SYY_SYY": np.sum(t * v * (Dyy * Dyy - (4 * d * Dyy + 2 * d * d))),
    }


def from_moments(a, b, d, dx, dy, t, wt, sg, wnu, nu, L):
    kc = 0.5 * (L - 1)
    s = np.arange(L) - kc
    U = [np.sum(t * s ** m) for m in range(5)]
    zxc, zyc = a * dx + b * (dy + kc), b * dx + d * (dy + kc)

    def N(p, q):
        V = U
        for _ in range(q):
            V = [zyc * V[m] + d * V[m + 1] for m in range(len(V) - 1)]
        for _ in range(p):
            V = [zxc * V[m] + b * V[m + 1] for m in range(len(V) - 1)]
        return V[0]

    e20, e11, e02 = N(2, 0) - a * N(0, 0), N(1, 1) - b * N(0, 0), N(0, 2) - d * N(0, 0)
    x2 = N(2, 1) - 2 * b * N(1, 0) - a * N(0, 1)
    x3 = N(1, 2) - d * N(1, 0) - 2 * b * N(0, 1)
    s3 = N(2, 2) - d * N(2, 0) - a * N(0, 2) - 4 * b * N(1, 1) + (a * d + 2 * b * b) * N(0, 0)
    v = wnu * nu
    return {
        "XX": wt * e20, "XY": wt * e11, "YY": wt * e02, "XF": sg * N(1, 0), "YF": sg * N(0, 1),
        "X_SXX": wnu * (N(3, 0) - 3 * a * N(1, 0)), "X_SXY": wnu * x2, "X_SYY": wnu * x3,
        "Y_SXX": wnu * x2, "Y_SXY": wnu * x3, "Y_SYY": wnu * (N(0, 3) - 3 * d * N(0, 1)),
        "F_SXX": sg * nu * e20, "F_SXY": sg * nu * e11, "F_SYY": sg * nu * e02,
        "SXX_SXX": v * (N(4, 0) - 6 * a * N(2, 0) + 3 * a * a * N(0, 0)),
        "SXX_SXY": v * (N(3, 1) - 3 * b * N(2, 0) - 3 * a * N(1, 1) + 3 * a * b * N(0, 0)),
        "SXX_SYY": v * s3, "SXY_SXY": v * s3,
        "SXY_SYY": v * (N(1, 3) - 3 * d * N(1, 1) - 3 * b * N(0, 2) + 3 * b * d * N(0, 0)),
        "SYY_SYY": v * (N(0, 4) - 6 * d * N(0, 2) + 3 * d * d * N(0, 0)),
    }


@pytest.mark.parametrize("L", [4, 8, 16])
def test_second_derivative_sums_from_row_moments(L):
    rng = np.random.default_rng(L)
    for _ in range(100):
        a, d = rng.uniform(0.02, 2.0, 2)
        b = rng.uniform(-0.95, 0.95) * np.sqrt(a * d)
        dx, dy = rng.uniform(-25, 25), rng.uniform(-40, 25)
        t = rng.normal(size=L) * np.exp(rng.normal(size=L))
        wt, wnu, nu = rng.uniform(0, 1), rng.uniform(0, 1), rng.uniform(0.1, 5)
        sg = rng.choice([-1.0, 1.0])
        ref = per_pixel(a, b, d, dx, dy, t, wt, sg, wnu, nu, L)
        got = from_moments(a, b, d, dx, dy, t, wt, sg, wnu, nu, L)
        j = dy + np.arange(L)
        zmax = np.max(np.abs(a * dx + b * j)) + np.max(np.abs(b * dx + d * j)) + a + abs(b) + d
        scale = np.sum(np.abs(t)) * max(1.0, zmax) ** 4
        for k in ref:
            assert abs(got[k] - ref[k]) <= 1e-12 * abs(ref[k]) + 1e-14 * scale, k
