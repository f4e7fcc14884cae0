"""Oracle Newton trust-region step for one source (TEST INFRASTRUCTURE ONLY).

Regier et al. 2018, Section IV-D: each source's parameters are optimised by Newton's
method with exact Hessians, step sizes controlled by a trust region (Nocedal & Wright);
Section VI-B: the trust-region subproblem is solved through an eigendecomposition.

Reading of the unstated details (shared with the device implementation as a reading,
not as code):
  * the step is taken in unconstrained coordinates: logit of q, frac_dev and the axis
    ratio; log of the radius and of every variance; identity for the rest;
  * the model minimised is f = -ELBO_s with gradient g and Hessian B in those
    coordinates (B includes the diagonal term g_theta * theta''(eta));
  * subproblem min g'p + p'Bp/2, |p| <= radius: the interior Newton step when B is
    positive definite and the step fits, else |p(mu)| = radius with
    p(mu) = -(B + mu I)^-1 g, mu > max(0, -lambda_min) (secular equation), and the hard
    case (g orthogonal to the lowest eigenspace) completed along that eigenvector;
  * ratio rho = actual / predicted increase: rho < 1/4 shrinks the radius by 4;
    rho > 3/4 with a boundary step doubles it (capped); the step is accepted when
    rho > eta_accept; a non-finite trial is rejected and shrinks the radius.
With the colour-prior mixture (43 parameters: the 16 responsibilities kappa, two
8-simplices) each simplex is mapped by a softmax with its last logit fixed at zero:
kappa_d = e^{eta_d} / (1 + sum_{e<7} e^{eta_e}) for d < 7 and kappa_7 = 1 / (1 + ...),
so the step is taken in 27 + 2 x 7 = 41 unconstrained coordinates; the Hessian there is
J^T (-H) J minus sum_i g_i (second derivative of theta_i in eta), with the Jacobian J of
theta(eta).
Gradient and Hessian come from the oracle's dual numbers; the eigendecomposition is
numpy's.
"""
import numpy as np

from . import oracle as O

LOGIT = {2, 3, 6}
LOG = {5} | {7 + 10 * t + o for t in (0, 1) for o in (1, 6, 7, 8, 9)}
NMIX = 8


def to_unconstrained(th):
    eta, d1, d2 = np.empty(27), np.empty(27), np.empty(27)
    for i in range(27):
        t = th[i]
        if i in LOGIT:
            eta[i] = np.log(t) - np.log1p(-t)
            d1[i] = t * (1 - t)
            d2[i] = d1[i] * (1 - 2 * t)
        elif i in LOG:
            eta[i] = np.log(t)
            d1[i] = t
            d2[i] = t
        else:
            eta[i], d1[i], d2[i] = t, 1.0, 0.0
    return eta, d1, d2


def from_unconstrained(eta):
    th = np.empty(27)
    for i in range(27):
        if i in LOGIT:
            th[i] = 1.0 / (1.0 + np.exp(-eta[i]))
        elif i in LOG:
            th[i] = np.exp(eta[i])
        else:
            th[i] = eta[i]
    return th


def softmax_block(kappa):
    """Unconstrained coordinates of one responsibility simplex: eta_d = log(kappa_d /
    kappa_7), d < 7; the Jacobian d kappa_d / d eta_e = kappa_d (delta_de - kappa_e)
    (delta_7e = 0), 8 x 7; and the second derivatives
    d2 kappa_d / d eta_e d eta_f = kappa_d [(delta_de - kappa_e)(delta_df - kappa_f)
    - kappa_e (delta_ef - kappa_f)], 8 x 7 x 7."""
    k = np.asarray(kappa, np.float64)
    eta = np.log(k[:NMIX - 1]) - np.log(k[NMIX - 1])
    D = np.zeros((NMIX, NMIX - 1))
    D[:NMIX - 1, :] = np.eye(NMIX - 1)
    A = D - k[None, :NMIX - 1]                       # delta_de - kappa_e
    J = k[:, None] * A
    kk = k[:NMIX - 1]
    T = k[:, None, None] * (A[:, :, None] * A[:, None, :]
                            - (kk[:, None] * (np.eye(NMIX - 1) - kk[None, :]))[None, :, :])
    return eta, J, T


def softmax_from_eta(eta):
    e = np.exp(np.concatenate([eta, [0.0]]))
    return e / e.sum()


def transform(row, npar):
    """Unconstrained coordinates of a source row with npar parameters (27, or 43 with the
    mixture responsibilities): (eta [m], J [npar x m], curvature(g) = sum_i g_i d2 theta_i /
    d eta^2 [m x m]) with m = 27 or 41."""
    eta27, d1, d2 = to_unconstrained(row[:27])
    if npar == 27:
        return eta27, np.diag(d1), lambda g, absolute=False: np.diag((np.abs(d2) if absolute else d2) * g[:27])
    m = 27 + 2 * (NMIX - 1)
    J = np.zeros((npar, m))
    J[:27, :27] = np.diag(d1)
    eta = np.zeros(m)
    eta[:27] = eta27
    blocks = []
    for t in range(2):
        et, Jt, Tt = softmax_block(row[27 + NMIX * t:27 + NMIX * (t + 1)])
        cs = slice(27 + (NMIX - 1) * t, 27 + (NMIX - 1) * (t + 1))
        eta[cs] = et
        J[27 + NMIX * t:27 + NMIX * (t + 1), cs] = Jt
        blocks.append((cs, slice(27 + NMIX * t, 27 + NMIX * (t + 1)), Tt))

    def curvature(g, absolute=False):
        f = np.abs if absolute else (lambda x: x)
        C = np.diag(np.concatenate([f(d2) * g[:27], np.zeros(m - 27)]))
        for cs, rs, Tt in blocks:
            C[cs, cs] += np.tensordot(g[rs], f(Tt), axes=1)
        return C

    return eta, J, curvature


def row_from_eta(eta, npar):
    """Inverse of transform: the npar parameters at unconstrained coordinates eta."""
    th = from_unconstrained(eta[:27])
    if npar == 27:
        return th
    ks = [softmax_from_eta(eta[27 + (NMIX - 1) * t:27 + (NMIX - 1) * (t + 1)]) for t in range(2)]
    return np.concatenate([th] + ks)


def subproblem(g, B, R):
    """Exact trust-region subproblem via the eigendecomposition of B."""
    lam, Q = np.linalg.eigh(0.5 * (B + B.T))
    gh = Q.T @ g
    lmin = lam.min()
    if lmin > 0:
        p = -gh / lam
        if p @ p <= R * R:
            return Q @ p, lam, gh, p
    lo0 = max(0.0, -lmin)
    tol = 1e-12 * max(np.abs(lam).max(), 1e-300)
    low = lam <= lmin + tol
    gmin2 = np.sum(gh[low] ** 2)
    rest = np.where(low, 0.0, gh / np.where(low, 1.0, lam + lo0))
    if lo0 > 0 and gmin2 <= 1e-28 * max(gh @ gh, 1e-300) and rest @ rest <= R * R:
        ph = -rest
        ph[np.argmin(lam)] = np.sqrt(max(R * R - rest @ rest, 0.0))
        return Q @ ph, lam, gh, ph

    def norm(mu):
        return np.linalg.norm(gh / (lam + mu))

    lo, hi = lo0, lo0 + np.linalg.norm(gh) / R
    mu = hi
    for _ in range(200):
        v = gh / (lam + mu)
        n2 = v @ v
        d3 = np.sum(v * v / (lam + mu))
        nrm = np.sqrt(n2)
        if abs(nrm - R) <= 1e-13 * R:
            break
        if nrm > R:
            lo = mu
        else:
            hi = mu
        nmu = mu + (nrm - R) / R * (n2 / d3)
        if not (lo < nmu < hi):
            nmu = 0.5 * (lo + hi)
        if nmu == mu:
            break
        mu = nmu
    ph = -gh / (lam + mu)
    return Q @ ph, lam, gh, ph


def source_fixed_elbo(f, theta_all, s, row):
    th = theta_all.copy()
    th[s, :len(row)] = row
    return O.source_elbo(O.Problem(f, th), s)


def n_params(f):
    return 43 if int(f.flags) & O.FLAG_MIX else 27


def newton_steps(f, theta_in, s, n_steps, radius0=1.0, radius_max=1e3, eta_accept=0.1, gtol=1e-8,
                 record=None):
    """n_steps trust-region iterations on source s, every other source fixed at theta_in.
    Returns (theta row [27 or 43], ELBO_s, radius)."""
    npar = n_params(f)
    row = theta_in[s, :npar].copy()
    R = radius0
    done = False
    f0 = None
    for _ in range(n_steps):
        if done:
            break
        th = theta_in.copy()
        th[s, :npar] = row
        P = O.Problem(f, th)
        val, g, gabs = O.source_grad(P, s)
        f0 = val[0] + val[1]
        H, Habs = O.source_hessian(P, s, with_abs=True)
        eta, J, curvature = transform(row, npar)
        gm = -J.T @ g
        B = -(J.T @ (0.5 * (H + H.T)) @ J) - curvature(g)
        if not np.max(np.abs(gm)) >= gtol:
            done = True
            break
        p, lam, gh, ph = subproblem(gm, B, R)
        pred = -np.sum(gh * ph + 0.5 * lam * ph * ph)
        pn = np.linalg.norm(ph)
        trial = row_from_eta(eta + p, npar)
        f1 = source_fixed_elbo(f, theta_in, s, trial)
        finite = np.isfinite(f1)
        rho = (f1 - f0) / pred if (finite and pred > 0) else -1.0
        Rold = R
        if not finite or rho < 0.25:
            R = 0.25 * R
        elif rho > 0.75 and pn >= 0.99 * Rold:
            R = min(2 * R, radius_max)
        if record is not None:
            record.append({"f0": f0, "f1": f1, "pred": pred, "rho": rho, "radius": Rold, "theta": row.copy(),
                           "grad": g, "gabs": gabs, "hess": H, "habs": Habs, "B": B, "g_eta": gm, "step": p})
        f_before = f0
        if finite and rho > eta_accept:
            row = trial
            f0 = f1
        if not (pred > 1e-15 * abs(f_before)) or R < 1e-12:
            done = True
    return row, f0, R
