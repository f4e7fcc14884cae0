"""Pins of the oracle trust-region step: optimality conditions of the subproblem
(Nocedal & Wright, Thm. 4.1), the coordinate transforms against finite differences,
and monotone ascent of the iterations."""
import numpy as np
import pytest

from oracle import newton as N


@pytest.mark.parametrize("seed", range(6))
def test_subproblem_satisfies_optimality_conditions(seed):
    rng = np.random.default_rng(seed)
    n = 27
    A = rng.standard_normal((n, n))
    B = 0.5 * (A + A.T)
    if seed % 2 == 0:
        B = B @ B.T / n + 0.1 * np.eye(n)       # positive definite
    g = rng.standard_normal(n)
    for R in (0.05, 1.0, 100.0):
        p, lam, gh, ph = N.subproblem(g, B, R)
        nrm = np.linalg.norm(p)
        assert nrm <= R * (1 + 1e-10)
        # (B + mu I) p = -g for some mu >= 0 with mu (R - |p|) = 0 and B + mu I PSD
        r = -g - B @ p
        mu = (r @ p) / (p @ p)
        assert mu >= -1e-9
        np.testing.assert_allclose(B @ p + mu * p, -g, atol=1e-8 * max(1.0, np.abs(g).max()))
        assert np.linalg.eigvalsh(B + mu * np.eye(n)).min() >= -1e-8
        if mu > 1e-8:
            assert abs(nrm - R) <= 1e-10 * R
        # no feasible point on a random sample does better
        m = lambda q: g @ q + 0.5 * q @ B @ q
        for _ in range(50):
            q = rng.standard_normal(n)
            q *= R * rng.random() / np.linalg.norm(q)
            assert m(q) >= m(p) - 1e-9 * max(1.0, abs(m(p)))


@pytest.mark.parametrize("seed", range(4))
def test_subproblem_hard_case(seed):
    """Hard case of the trust-region subproblem (Nocedal & Wright, Section 4.3): B has a
    negative lowest eigenvalue lambda_1 and g is orthogonal to its eigenvector q_1, and the
    radius exceeds |(B - lambda_1 I)^+ g|.  Then mu = -lambda_1 and the solution is that
    pseudo-inverse step completed along q_1 to the boundary: |p| = R, (B + mu I) p = -g,
    B + mu I positive semidefinite, and q_1^T p = +-sqrt(R^2 - |rest|^2)."""
    rng = np.random.default_rng(100 + seed)
    n = 27
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.sort(rng.uniform(-2.0, 5.0, n))
    lam[0] = -3.0 - seed                              # simple, negative lowest eigenvalue
    B = (Q * lam) @ Q.T
    gh = rng.standard_normal(n)
    gh[0] = 0.0                                       # g orthogonal to q_1
    g = Q @ gh
    rest = gh[1:] / (lam[1:] - lam[0])                # |(B - lambda_1 I)^+ g| in the eigenbasis
    R = 1.5 * np.linalg.norm(rest) + 0.1 * seed
    p, *_ = N.subproblem(g, B, R)
    assert abs(np.linalg.norm(p) - R) <= 1e-12 * R
    mu = -lam[0]
    np.testing.assert_allclose(B @ p + mu * p, -g, atol=1e-10 * max(1.0, np.abs(g).max()))
    assert np.linalg.eigvalsh(B + mu * np.eye(n)).min() >= -1e-10
    tau = np.sqrt(R * R - rest @ rest)
    np.testing.assert_allclose(abs(Q[:, 0] @ p), tau, rtol=1e-10)
    # the component orthogonal to q_1 is -(B - lambda_1 I)^+ g
    np.testing.assert_allclose(Q[:, 1:].T @ p, -rest, rtol=1e-10, atol=1e-12 * R)
    # the model value is the global minimum over the ball: -sum over the eigenbasis
    m = lambda q: g @ q + 0.5 * q @ B @ q
    best = -0.5 * np.sum(gh[1:] ** 2 * (lam[1:] + 2 * mu) / (lam[1:] + mu) ** 2) + 0.5 * lam[0] * tau ** 2
    np.testing.assert_allclose(m(p), best, rtol=1e-10)
    for _ in range(200):
        q = rng.standard_normal(n)
        q *= R * rng.random() ** (1.0 / n) / np.linalg.norm(q)
        assert m(q) >= m(p) - 1e-9 * abs(m(p))


def test_transforms_round_trip_and_derivatives():
    rng = np.random.default_rng(0)
    th = np.abs(rng.uniform(0.1, 0.9, 27))
    th[[0, 1, 4]] = [3.0, -2.0, 0.7]
    eta, d1, d2 = N.to_unconstrained(th)
    np.testing.assert_allclose(N.from_unconstrained(eta), th, rtol=1e-14)
    h = 1e-5
    for i in range(27):
        e1, e2 = eta.copy(), eta.copy()
        e1[i] += h
        e2[i] -= h
        fd1 = (N.from_unconstrained(e1)[i] - N.from_unconstrained(e2)[i]) / (2 * h)
        fd2 = (N.from_unconstrained(e1)[i] - 2 * th[i] + N.from_unconstrained(e2)[i]) / h ** 2
        np.testing.assert_allclose(d1[i], fd1, rtol=1e-8, atol=1e-12)
        np.testing.assert_allclose(d2[i], fd2, rtol=1e-4, atol=1e-6)


def test_iterations_ascend(synth, O):
    f = synth.tiny(S=2, n_bands=2, size=17, side=11, seed=8)
    rec = []
    row, fend, R = N.newton_steps(f, f.theta, 0, 8, record=rec)
    start = O.source_elbo(O.Problem(f), 0)
    assert fend >= start
    cur = start
    for r in rec:
        if r["rho"] > 0.1:
            assert r["f1"] > cur
            cur = r["f1"]
    th = f.theta.copy()
    th[0, :27] = row
    np.testing.assert_allclose(O.source_elbo(O.Problem(f, th), 0), fend, rtol=1e-13)


def test_softmax_transform_derivatives_and_round_trip():
    """Responsibilities through the softmax with the last logit fixed at 0: round trip,
    the Jacobian and second derivatives against finite differences, rows of J summing to
    zero over the simplex (the sum stays 1)."""
    rng = np.random.default_rng(1)
    k = rng.dirichlet(np.ones(8))
    eta, J, T = N.softmax_block(k)
    np.testing.assert_allclose(N.softmax_from_eta(eta), k, rtol=1e-14)
    np.testing.assert_allclose(J.sum(0), 0.0, atol=1e-16)
    h = 1e-5
    for e in range(7):
        ep, em = eta.copy(), eta.copy()
        ep[e] += h
        em[e] -= h
        fd = (N.softmax_from_eta(ep) - N.softmax_from_eta(em)) / (2 * h)
        np.testing.assert_allclose(J[:, e], fd, rtol=1e-8, atol=1e-12)
        h = 1e-4   # second differences: rounding ~ eps / h^2, truncation ~ h^2
        for g in range(7):
            e2 = [eta.copy() for _ in range(4)]
            e2[0][[e, g]] += h
            e2[1][e] += h
            e2[1][g] -= h
            e2[2][e] -= h
            e2[2][g] += h
            e2[3][[e, g]] -= h
            if e == g:
                fd2 = (N.softmax_from_eta(eta + np.eye(7)[e] * 2 * h) - 2 * k
                       + N.softmax_from_eta(eta - np.eye(7)[e] * 2 * h)) / (4 * h * h)
            else:
                fd2 = (N.softmax_from_eta(e2[0]) - N.softmax_from_eta(e2[1]) - N.softmax_from_eta(e2[2])
                       + N.softmax_from_eta(e2[3])) / (4 * h * h)
            np.testing.assert_allclose(T[:, e, g], fd2, rtol=1e-5, atol=1e-7)
        h = 1e-5


def test_mixture_iterations_ascend_and_stay_on_the_simplex(synth, O):
    f = synth.with_color_mixture(synth.tiny(S=2, n_bands=2, size=17, side=11, seed=9), seed=6)
    rec = []
    row, fend, R = N.newton_steps(f, f.theta, 0, 6, record=rec)
    assert row.shape == (43,)
    start = O.source_elbo(O.Problem(f), 0)
    assert fend > start
    np.testing.assert_allclose([row[27:35].sum(), row[35:43].sum()], 1.0, rtol=1e-14)
    assert np.all(row[27:43] > 0)
    assert any(np.any(r["theta"][27:43] != f.theta[0, 27:43]) for r in rec[1:])
    th = f.theta.copy()
    th[0, :43] = row
    np.testing.assert_allclose(O.source_elbo(O.Problem(f, th), 0), fend, rtol=1e-13)
