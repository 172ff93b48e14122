"""Pins for the control logic of the oracle's MDOT (Alg. 1) and
TruncatedNewtonProject (Alg. 4) drivers (no GPU).

Every end-to-end pin of the solver holds for any temperature schedule,
because the solution at the final temperature is unique. These tests check
the schedule itself, against things other than the oracle's own code:

* fixed decay factor: the inverse temperatures are beta_i q^k capped at
  beta_f, and the number of MDOT steps is the closed form
  ceil(log_q(beta_f / beta_i)) + 1;
* AdjustSchedule (Sec. 3.3) and the forcing term (Alg. 4) against
  hand-worked values of the printed rules (tests/golden/alg1_rules.json),
  and every decay factor a solve reaches lies in {2^(2^-k)};
* the extrapolation of Alg. 1: exact for potentials affine in beta, and on a
  separable cost with uniform marginals -- whose projected potentials are
  affine in beta -- every extrapolated start is already projected, so no
  ChiSinkhorn sweep or Newton step runs after the first temperature;
* smoothing (Sec. 3.4) and eps_d (Alg. 1): at every intermediate
  temperature the projected plan, evaluated densely here, has row marginals
  (1 - w_r eps_d) r + w_r eps_d / n and column marginals within eps_d / 2 of
  (1 - w_c eps_d) c + w_c eps_d / m, with eps_d = min(H(r), H(c)) / beta^p
  computed from SciPy's entropy (a rectangular instance, so 1/n and 1/m
  cannot be swapped unnoticed);
* the warm discount (App. B): each NewtonSolve starts from the second last
  level 1 - 4^-(J-1) of the previous one (levels 1 - 4^-J), or 0;
* the CG tolerance eta/4 of Alg. 2: a NewtonSolve capped at one discount
  level stops its CG at the first iteration whose residual, recomputed
  densely here, is at most (eta/4) |grad g|_1, on cases where eta/2 would
  stop earlier;
* resuming a solve from its saved state reproduces the uninterrupted solve
  bit for bit, and a warm start at the solution needs no Newton step.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.stats import entropy

import oracle as O
from paper_2504_02067_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rules():
    with open(os.path.join(GOLDEN, "alg1_rules.json")) as fh:
        return json.load(fh)


def _rect_problem(seed=11, n=48, m=64):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, size=(n, 2))
    Y = rng.uniform(0.0, 1.0, size=(m, 2))
    r = W.dirichlet_marginal(rng, n)
    c = W.dirichlet_marginal(rng, m)
    return W.sqeuclid_cost(X, Y), r, c


# ---------------------------------------------------------------- schedule

@pytest.mark.parametrize("q1", [2.0, 4.0, math.sqrt(2.0)])
def test_fixed_decay_factor_gives_geometric_schedule(q1):
    p = W.small_points_problem(1000)
    u, v, st, tr, _ = O.solve_ex(p.C, p.r, p.c, gamma_init=p.gamma_init,
                                 gamma_final=p.gamma_final, tol=p.tol, adaptive_q=0, q1=q1)
    assert st["status"] == 0
    bi, bf = 1.0 / p.gamma_init, 1.0 / p.gamma_final
    steps = math.ceil(math.log(bf / bi) / math.log(q1) - 1e-12) + 1
    assert st["mdot_steps"] == steps == tr["n_steps"]
    want = [min(bi * q1 ** k, bf) for k in range(steps)]
    np.testing.assert_allclose(tr["beta"], want, rtol=1e-13, atol=0)
    assert tr["beta"][-1] == bf
    assert np.all(tr["q"] == q1)


def test_adjust_schedule_matches_hand_worked_sequence():
    g = _rules()["adjust_schedule"]
    q = g["q0"]
    for d, want in zip(g["delta_min"], g["q"]):
        q = O.adjust_schedule(q, d)
        assert q == pytest.approx(want, rel=1e-15, abs=0)


def test_forcing_term_matches_hand_worked_values():
    for gnorm, eps, want in _rules()["forcing_eta"]["cases"]:
        assert O.forcing_eta(gnorm, eps) == pytest.approx(want, rel=1e-15)


@pytest.mark.parametrize("side,kind,seed", [(10, "sqeuclid", 2000), (12, "sqeuclid", 2001),
                                            (12, "l1", 2000)])
def test_adaptive_schedule_follows_adjust_schedule(side, kind, seed):
    p = W.grid_blob_problem(side, seed, kind)
    u, v, st, tr, _ = O.solve_ex(p.C.astype(np.float64), p.r, p.c, gamma_init=p.gamma_init,
                                 gamma_final=p.gamma_final, tol=p.tol)
    assert st["status"] == 0
    beta, q, dmin = tr["beta"], tr["q"], tr["delta_min"]
    bf = 1.0 / p.gamma_final
    qprev = 2.0
    for t in range(len(beta)):
        last = t == len(beta) - 1
        want_q = qprev if last else O.adjust_schedule(qprev, dmin[t])
        assert q[t] == want_q
        if not last:
            assert beta[t + 1] == min(q[t] * beta[t], bf)
        # every reachable decay factor is 2^(2^-k): log2(log2(q)) is an integer
        k = math.log2(math.log2(q[t]))
        assert abs(k - round(k)) < 1e-9 and round(k) <= 0
        qprev = q[t]
    # the schedule did adapt on these instances (both branches of the rule)
    assert len(set(np.round(q, 12))) >= 2


# ---------------------------------------------------------------- extrapolation

def test_extrapolation_exact_on_affine_potentials():
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal(7), rng.standard_normal(7)
    b0, b1, b2 = 3.0, 6.0, 9.5
    z, zp = O.extrapolate(a + b * b1, a + b * b0, b0, b1, b2)
    np.testing.assert_allclose(z, a + b * b2, rtol=1e-14, atol=1e-13)
    np.testing.assert_array_equal(zp, a + b * b1)
    # first step: beta_prev = 0 extrapolates from z^(0) through the origin of beta
    z, _ = O.extrapolate(a + b * b1, a, 0.0, b1, b2)
    np.testing.assert_allclose(z, a + b * b2, rtol=1e-14, atol=1e-13)


@pytest.mark.parametrize("q1,adaptive", [(2.0, 1), (2.0, 0), (4.0, 0)])
def test_extrapolated_starts_are_projected_on_separable_costs(q1, adaptive):
    rng = np.random.default_rng(21)
    n, m = 40, 56
    a = rng.uniform(0.0, 0.5, n)
    b = rng.uniform(0.0, 0.5, m)
    C = a[:, None] + b[None, :]
    r = np.full(n, 1.0 / n)
    c = np.full(m, 1.0 / m)
    u, v, st, tr, _ = O.solve_ex(C, r, c, gamma_init=0.1, gamma_final=1e-3, tol=1e-9,
                                 q1=q1, adaptive_q=adaptive)
    assert st["status"] == 0 and tr["n_steps"] >= 4
    assert tr["start_err"][0] > 0.1          # the first start is far from the projection
    assert np.all(tr["start_err"][1:] < 1e-12)
    assert np.all(tr["sweeps"][1:] == 0) and np.all(tr["newton"][1:] == 0)
    # the plan is the independent coupling r c^T (separable cost)
    P = np.exp(u[:, None] + v[None, :] - C / 1e-3)
    np.testing.assert_allclose(P, np.outer(r, c), rtol=1e-9)


# ---------------------------------------------------------------- smoothing, eps_d

def test_projections_hit_smoothed_marginals_within_half_eps():
    C, r, c = _rect_problem()
    n, m = C.shape
    w_r, p_exp, tol = 0.45, 1.5, 1e-9
    u, v, st, tr, _ = O.solve_ex(C, r, c, gamma_init=0.1, gamma_final=1e-3, tol=tol,
                                 potentials=True)
    assert st["status"] == 0
    hmin = min(entropy(r), entropy(c))
    for t, beta in enumerate(tr["beta"]):
        last = t == tr["n_steps"] - 1
        eps = hmin / beta ** p_exp
        if last:
            eps = min(eps, tol / 2)
        assert tr["eps_d"][t] == pytest.approx(eps, rel=1e-13)
        rt = (1 - w_r * eps) * r + w_r * eps / n
        ct = (1 - (0.5 - w_r) * eps) * c + (0.5 - w_r) * eps / m
        P = np.exp(tr["u_proj"][t][:, None] + tr["v_proj"][t][None, :] - beta * C)
        # the closing row fit makes the rows exact; the columns stay within eps_d / 2
        assert np.abs(P.sum(1) - rt).sum() <= 1e-13
        assert np.abs(P.sum(0) - ct).sum() <= eps / 2 * (1 + 1e-9)
        if not last:
            # smoothing moved the targets by far more than the tolerance checked above
            assert np.abs(rt - r).sum() > 1e3 * 1e-13
    assert st["err_r"] + st["err_c"] <= tol


# ---------------------------------------------------------------- warm discount

def _level(rho):
    """J with rho = 1 - 4^-J (rho = 0 is J = 0)."""
    if rho == 0.0:
        return 0
    j = -math.log(1.0 - rho, 4)
    assert abs(j - round(j)) < 1e-9, rho
    return int(round(j))


def test_discount_levels_match_hand_worked_values():
    g = _rules()["discount_levels"]
    for k, lev in enumerate(g["levels"]):
        assert _level(lev) == k
    for rho_out, nxt in g["next_start"]:
        J = _level(rho_out)
        assert (1.0 - 4.0 ** -(J - 1) if J >= 2 else 0.0) == nxt


@pytest.mark.parametrize("adaptive", [1, 0])
def test_newton_solves_start_from_second_last_level(adaptive):
    p = W.small_points_problem(1001)
    u, v, st, tr, _ = O.solve_ex(p.C, p.r, p.c, gamma_init=p.gamma_init,
                                 gamma_final=p.gamma_final, tol=p.tol, adaptive_rho0=adaptive)
    assert st["status"] == 0 and tr["n_newton"] >= 5
    rho0, rho_out, levels = tr["rho0"], tr["rho_out"], tr["levels"]
    assert rho0[0] == 0.0
    for k in range(len(rho0)):
        J0, J1 = _level(rho0[k]), _level(rho_out[k])
        assert J1 == J0 + levels[k]              # one level per discount solved
        if k + 1 < len(rho0):
            want = (1.0 - 4.0 ** -(J1 - 1) if J1 >= 2 else 0.0) if adaptive else 0.0
            assert rho0[k + 1] == want
    if adaptive:
        assert max(rho0) >= 0.75                # the warm discount was exercised


# ---------------------------------------------------------------- CG tolerance eta / 4

def _dense_pcg_first_hit(F, M, b, tol, kmax):
    """Textbook Jacobi-preconditioned CG from 0 on F d = b; the first
    iteration whose L1 residual is <= tol."""
    d = np.zeros_like(b)
    res = b.copy()
    z = res / M
    p = z.copy()
    rz = res @ z
    for k in range(1, kmax + 1):
        q = F @ p
        alpha = rz / (p @ q)
        d = d + alpha * p
        res = res - alpha * q
        if np.abs(res).sum() <= tol:
            return k, d
        z = res / M
        rz_new = res @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return None, d


@pytest.mark.parametrize("seed", range(6))
def test_cg_in_newton_solve_stops_at_quarter_eta(seed):
    rng = np.random.default_rng(300 + seed)
    n, m = 24, 30
    C = rng.uniform(0.0, 1.0, (n, m))
    r = W.dirichlet_marginal(rng, n)
    c = W.dirichlet_marginal(rng, m)
    beta, rho = 8.0, 0.9375
    u = np.log(r) + 0.3 * rng.standard_normal(n)
    v = np.log(c) - O.log_col_marginal(C, beta, u, np.zeros(m))        # c(P) = c
    P = np.exp(u[:, None] + v[None, :] - beta * C)
    rP = P.sum(1)
    grad = rP - r
    gn = np.abs(grad).sum()
    F = np.diag(rP) - rho * (P / c[None, :]) @ P.T
    s = ((P * P) / c[None, :]).sum(1)
    M = np.maximum(rP - rho * s, (1.0 - rho) * rP)
    # the rho = 0 direction must fail the forcing test, so that one CG solve runs
    F1 = np.diag(rP) - (P / c[None, :]) @ P.T
    e0 = np.abs(F1 @ (-grad / rP) + grad).sum() / gn
    # pick eta so that eta/4 and eta/2 are first reached at different iterations
    chosen = None
    for eta in np.geomspace(0.99 * min(e0, 1.0), 1e-6, 200):
        k4, d4 = _dense_pcg_first_hit(F, M, -grad, eta / 4 * gn, 200)
        k2, _ = _dense_pcg_first_hit(F, M, -grad, eta / 2 * gn, 200)
        if k4 is not None and k2 is not None and k4 > k2 >= 1:
            chosen = (eta, k4, d4)
            break
    assert chosen is not None
    eta, k4, d4 = chosen
    res = O.newton_solve(C, beta, u, v, r, c, np.log(rP), eta, rho0=rho, max_levels=1)
    assert res.levels == 1
    assert res.cg_iters == k4
    np.testing.assert_allclose(res.du, d4, rtol=1e-9, atol=1e-12)
    assert np.abs(F @ res.du + grad).sum() <= eta / 4 * gn * (1 + 1e-9)


# ---------------------------------------------------------------- state, warm start

@pytest.mark.parametrize("stop_after", [1, 3, 6])
def test_resume_from_saved_state_is_bitwise(stop_after):
    p = W.small_points_problem(1002)
    kw = dict(gamma_init=p.gamma_init, gamma_final=p.gamma_final, tol=p.tol)
    u0, v0, st0, tr0, _ = O.solve_ex(p.C, p.r, p.c, **kw)
    assert st0["status"] == 0 and st0["mdot_steps"] > stop_after
    _, _, st1, tr1, state = O.solve_ex(p.C, p.r, p.c, max_mdot=stop_after, **kw)
    assert st1["status"] == 4                   # stopped by the MDOT step cap
    assert state["t"] == stop_after + 1
    u2, v2, st2, tr2, _ = O.solve_ex(p.C, p.r, p.c, resume=state, **kw)
    assert st2["status"] == 0
    np.testing.assert_array_equal(u2, u0)
    np.testing.assert_array_equal(v2, v0)
    assert list(tr1["beta"]) + list(tr2["beta"]) == list(tr0["beta"])
    assert st1["newton_steps"] + st2["newton_steps"] == st0["newton_steps"]


def test_warm_start_at_the_solution_takes_no_newton_step():
    p = W.small_points_problem(1000)
    kw = dict(gamma_init=p.gamma_final, gamma_final=p.gamma_final, tol=p.tol)
    u0, v0, st0, _, _ = O.solve_ex(p.C, p.r, p.c, gamma_init=p.gamma_init,
                                   gamma_final=p.gamma_final, tol=p.tol)
    u1, v1, st1, tr1, _ = O.solve_ex(p.C, p.r, p.c, warm=(u0, v0), **kw)
    assert st1["status"] == 0 and tr1["n_steps"] == 1
    assert st1["newton_steps"] == 0 and st1["sinkhorn_iters"] == 0
    assert abs(st1["cost"] - st0["cost"]) <= 1e-12 * st0["cost"]
    # a cold start at the same single temperature needs Newton steps
    _, _, st2, _, _ = O.solve_ex(p.C, p.r, p.c, **kw)
    assert st2["newton_steps"] > 0


# ---------------------------------------------------------------- ChiSinkhorn tolerance

def _chi_sweeps(C, beta, u, r, c, eps_chi, kmax=10000):
    """Sweeps of Alg. 3 (row fit, column fix, row refresh) from the column-fixed
    start until chi^2(r | r(P)) <= eps_chi, with the plan formed densely."""
    def colfix(u):
        x = u[:, None] - beta * C
        mx = x.max(0)
        return np.log(c) - (mx + np.log(np.exp(x - mx).sum(0)))

    v = colfix(u)
    rP = np.exp(u[:, None] + v[None, :] - beta * C).sum(1)
    for k in range(kmax):
        if ((r - rP) ** 2 / rP).sum() <= eps_chi:
            return k
        u = u + np.log(r) - np.log(rP)
        v = colfix(u)
        rP = np.exp(u[:, None] + v[None, :] - beta * C).sum(1)
    return None


@pytest.mark.parametrize("seed", range(3))
def test_chi_sinkhorn_inside_tnp_stops_at_eps_two_fifths(seed):
    rng = np.random.default_rng(700 + seed)
    n, m = 20, 28
    C = rng.uniform(0.0, 1.0, (n, m))
    r = W.dirichlet_marginal(rng, n)
    c = W.dirichlet_marginal(rng, m)
    beta = 30.0
    u0 = np.log(r) + 2.0 * rng.standard_normal(n)
    chosen = None
    for eps in np.geomspace(1e-2, 1e-9, 120):
        k4 = _chi_sweeps(C, beta, u0, r, c, eps ** 0.4)
        k5 = _chi_sweeps(C, beta, u0, r, c, eps ** 0.5)
        if k4 is not None and k5 is not None and k5 > k4 >= 1:
            chosen = (eps, k4)
            break
    assert chosen is not None
    eps, k4 = chosen
    opts = O.default_opts(max_newton=1)
    _, _, _, _, st, status = O.tnp(C, beta, u0, np.zeros(m), r, c, eps, opts=opts)
    assert st["sinkhorn_iters"] == k4
