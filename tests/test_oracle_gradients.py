"""Pins of the oracle's derivative formulas (oracle/gradients.py) against
central finite differences of fully converged entropic OT solutions.

The solutions come from a plain log-domain Sinkhorn written here (alternating
exact row and column fits until both marginal errors are below 1e-15), not
from the oracle's solver, so a dropped term, a wrong sign or a transposed
operand in the formulas shows up as a finite-difference mismatch.
"""
import numpy as np
import pytest
from scipy.special import logsumexp

from oracle import gradients as OG

GAMMA = 0.1
BETA = 1.0 / GAMMA


def sinkhorn(C, r, c, beta=BETA, iters=20000):
    n, m = C.shape
    u = np.zeros(n); v = np.zeros(m)
    lr, lc = np.log(r), np.log(c)
    for _ in range(iters):
        u = lr - logsumexp(v[None, :] - beta * C, axis=1)
        v = lc - logsumexp(u[:, None] - beta * C, axis=0)
        P = np.exp(u[:, None] + v[None, :] - beta * C)
        if np.abs(P.sum(1) - r).sum() < 1e-15:
            break
    return u, v


def W_of(C, r, c):
    u, v = sinkhorn(C, r, c)
    return OG.value(C, BETA, u, v, r, c)


def S_of(C, r, c):
    u, v = sinkhorn(C, r, c)
    return (OG.plan(C, BETA, u, v) * C).sum()


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(12)
    n, m = 7, 9
    C = rng.uniform(0, 1, size=(n, m))
    r = rng.dirichlet(np.ones(n)) + 0.05; r /= r.sum()
    c = rng.dirichlet(np.ones(m)) + 0.05; c /= c.sum()
    u, v = sinkhorn(C, r, c)
    return C, r, c, u, v


def test_sinkhorn_helper_converged(case):
    C, r, c, u, v = case
    P = OG.plan(C, BETA, u, v)
    assert np.abs(P.sum(1) - r).sum() < 1e-14 and np.abs(P.sum(0) - c).sum() < 1e-14


@pytest.mark.parametrize("w_W,w_S", [(1.0, 0.0), (0.0, 1.0), (0.7, -1.3)])
def test_cost_cotangent_matches_finite_differences(case, w_W, w_S):
    C, r, c, u, v = case
    G, _, _, _, _, _ = OG.vjp(C, BETA, u, v, w_W, w_S)
    h = 1e-6
    for (i, j) in [(0, 0), (3, 5), (6, 8), (2, 1)]:
        E = np.zeros_like(C); E[i, j] = h
        fd = (w_W * (W_of(C + E, r, c) - W_of(C - E, r, c))
              + w_S * (S_of(C + E, r, c) - S_of(C - E, r, c))) / (2 * h)
        assert fd == pytest.approx(G[i, j], rel=1e-6, abs=1e-10)


@pytest.mark.parametrize("w_W,w_S", [(1.0, 0.0), (0.0, 1.0)])
def test_marginal_gradients_match_finite_differences(case, w_W, w_S):
    C, r, c, u, v = case
    _, gr, gc, _, _, _ = OG.vjp(C, BETA, u, v, w_W, w_S)
    assert abs(gr.sum()) < 1e-12 and abs(gc.sum()) < 1e-12
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(3):
        dr = rng.standard_normal(r.size); dr -= dr.mean()        # stays on the simplex
        dc = rng.standard_normal(c.size); dc -= dc.mean()
        fd = 0.0
        if w_W:
            fd += w_W * (W_of(C, r + h * dr, c + h * dc) - W_of(C, r - h * dr, c - h * dc)) / (2 * h)
        if w_S:
            fd += w_S * (S_of(C, r + h * dr, c + h * dc) - S_of(C, r - h * dr, c - h * dc)) / (2 * h)
        assert fd == pytest.approx(gr @ dr + gc @ dc, rel=1e-6, abs=1e-10)


def test_points_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    n, m, d = 6, 8, 3
    X = rng.standard_normal((n, d)); Y = rng.standard_normal((m, d))
    s = 9.0
    r = np.full(n, 1.0 / n); c = np.full(m, 1.0 / m)

    def cost(X, Y):
        return ((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1) / s

    def L(X, Y):
        C = cost(X, Y)
        u, v = sinkhorn(C, r, c)
        return 0.4 * OG.value(C, BETA, u, v, r, c) + 1.1 * (OG.plan(C, BETA, u, v) * C).sum()

    C = cost(X, Y)
    u, v = sinkhorn(C, r, c)
    G, *_ = OG.vjp(C, BETA, u, v, 0.4, 1.1)
    gX, gY = OG.points_grad(X, Y, s, G)
    h = 1e-6
    for (i, k) in [(0, 0), (4, 2), (5, 1)]:
        E = np.zeros_like(X); E[i, k] = h
        assert (L(X + E, Y) - L(X - E, Y)) / (2 * h) == pytest.approx(gX[i, k], rel=1e-6, abs=1e-10)
    for (j, k) in [(0, 1), (7, 2)]:
        E = np.zeros_like(Y); E[j, k] = h
        assert (L(X, Y + E) - L(X, Y - E)) / (2 * h) == pytest.approx(gY[j, k], rel=1e-6, abs=1e-10)


def test_hessian_solve_gauge_and_residual(case):
    C, r, c, u, v = case
    P = OG.plan(C, BETA, u, v)
    a = (P * C).sum(1); b = (P * C).sum(0)
    lam, mu = OG.hessian_solve(P, a, b)
    np.testing.assert_allclose(P.sum(1) * lam + P @ mu, a, atol=1e-14)
    np.testing.assert_allclose(P.T @ lam + P.sum(0) * mu, b, atol=1e-14)
    # the gauge (lam + t, mu - t) leaves lam_i + mu_j unchanged
    G1, *_ = OG.vjp(C, BETA, u, v, 0.0, 1.0)
    lam2, mu2 = lam + 0.3, mu - 0.3
    G2 = P * (1.0 + BETA * (lam2[:, None] + mu2[None, :] - C))
    np.testing.assert_allclose(G1, G2, atol=1e-14)
