"""GPU against the oracle, step by step: the decisions of Alg. 1 (MDOT:
eps_d, smoothing, AdjustSchedule, extrapolation) and of Alg. 4 (forcing
term, CG tolerance eta/4, warm discount of App. B, line search, row refresh)
recorded by eot_solve_ex and by the oracle's traced solve on the same input.
The oracle's rules are pinned on their own in tests/test_oracle_alg1_pins.py;
here the GPU path must take the same steps. Also the carried state of
Alg. 1: a solve stopped after k temperatures and resumed equals the
uninterrupted solve bitwise, and its saved state equals the oracle's; and a
warm start from given potentials takes the oracle's steps.

Tolerances: integer decisions (Newton steps, sweeps, CG iterations, discount
levels) and the schedule (beta, q, alpha, rho) exactly equal; L1 errors within
1e-12 absolute + 1e-8 relative (sums of cancelling FP64 terms whose summation
order differs); the forcing term eta = max(g, 0.8 eps / g) and the CG
tolerance eta g / 4 inherit the relative error of g = ||grad g||_1, so they are
compared relative to 1e-8 + 1e-12 / g (twice that for the CG tolerance);
potentials 1e-10 relative to their scale. The line search's step length is
compared exactly while ||grad g||_1 >= 1e-7; below that, Armijo's test on the
FP64 mass is decided by rounding on both sides. One exception: a NewtonSolve that
ends at the discount cap 1 - 2^-30 (the forcing miss of nearly decomposable
plans) runs its last CG solves at a condition number up to ~2e9, where the
iteration count depends on rounding; for those Newton steps the CG count is
compared within 25%, and from that Newton step on the two trajectories are
only as close as those CG solves (tolerance eta g / 4): the L1 errors of later
steps are compared within 1e-2 relative. Before it, the potentials of the two
sides agree to ~1e-12 relative along the whole trajectory, so an L1 marginal
error (n terms r_i - r(P)_i) is compared within 1e-11 absolute."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2504_02067_amd import eot
from paper_2504_02067_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

EXACT = ("newton", "sweeps", "step_of", "levels", "beta", "q", "rho0", "rho_out")
# Armijo's test on the mass (mass - 1 <= 0.99 alpha slope) is decided by rounding
# once |slope| ~ sum grad^2 / r(P) falls below the ~1e-15 rounding of the FP64
# mass (each side sums the plan with its own exp): below this gradient norm the
# two sides may accept different step lengths
ALPHA_DECIDABLE = 1e-7
CLOSE = ("eps_d", "start_err", "gnorm", "gnorm_next")
RHO_CAP = 1.0 - 2.0 ** -30


def say(msg):
    print(f"[gpu-trace] {msg}", flush=True)


def dvec(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def _opts(p, **kw):
    return dict(gamma_init=p.gamma_init, gamma_final=p.gamma_final, tol=p.tol, **kw)


def _close(a, b, rtol, atol, where):
    bad = np.abs(a - b) > atol + rtol * np.abs(b)
    assert not bad.any(), (where, np.nonzero(bad)[0], a[bad], b[bad])


def compare_traces(tg, to, where):
    assert tg["n_steps"] == to["n_steps"], (where, tg["n_steps"], to["n_steps"])
    assert tg["n_newton"] == to["n_newton"], (where, tg["n_newton"], to["n_newton"])
    for k in EXACT:
        np.testing.assert_array_equal(tg[k], to[k], err_msg=f"{where}: {k}")
    dec = to["gnorm"] >= ALPHA_DECIDABLE
    np.testing.assert_array_equal(tg["alpha"][dec], to["alpha"][dec], err_msg=f"{where}: alpha")
    # the trajectories part where a capped NewtonSolve ran or an undecidable
    # line search went different ways; from there on only the loose checks apply
    capped = to["rho_out"] > RHO_CAP
    parted = capped | (tg["alpha"] != to["alpha"])
    kc = int(np.argmax(parted)) if parted.any() else len(parted)
    tc = int(to["step_of"][kc]) if parted.any() else len(to["beta"]) + 1
    tight = np.arange(len(capped)) <= kc                            # its own gnorm still tight
    steps_tight = np.arange(1, len(to["beta"]) + 1) <= tc
    _close(tg["eps_d"], to["eps_d"], 1e-12, 0.0, f"{where}: eps_d")
    for k, idx, loose in (("start_err", steps_tight, ~steps_tight), ("gnorm", tight, ~tight),
                          ("gnorm_next", np.arange(len(capped)) < kc,
                           np.arange(len(capped)) >= kc)):
        _close(tg[k][idx], to[k][idx], 1e-8, 1e-11, f"{where}: {k}")
        if k == "gnorm_next":
            # after the parting: close, or both already below the projection's tolerance
            eps_t = 0.5 * to["eps_d"][to["step_of"] - 1]
            a, b = tg[k][loose], to[k][loose]
            ok = (np.abs(a - b) <= 1e-2 * np.abs(b) + 1e-11) | ((a <= eps_t[loose]) & (b <= eps_t[loose]))
            assert ok.all(), (where, k, np.nonzero(loose)[0][~ok], a[~ok], b[~ok])
        else:
            _close(tg[k][loose], to[k][loose], 1e-2, 1e-11, f"{where}: {k} (after the parting)")
    g = to["gnorm"]
    for k, mult in (("eta", 1.0), ("cg_tol", 2.0)):
        rel = np.abs(tg[k] - to[k]) / to[k]
        lim = np.where(tight, mult * (1e-8 + 1e-11 / g), 2e-2)
        bad = rel > lim
        assert not bad.any(), (where, k, np.nonzero(bad)[0], rel[bad], g[bad])
    np.testing.assert_array_equal(tg["cg_iters"][:kc], to["cg_iters"][:kc],
                                  err_msg=f"{where}: cg_iters before the first capped step")
    a, b = tg["cg_iters"][kc:], to["cg_iters"][kc:]
    assert (np.abs(a - b) <= 0.25 * b).all(), (where, a, b)
    # delta_min: +inf (no Newton step) in the same places, values close
    a, b = tg["delta_min"], to["delta_min"]
    assert np.array_equal(np.isinf(a), np.isinf(b)), where
    fin = np.isfinite(a)
    before = np.arange(1, len(to["beta"]) + 1) < tc                 # steps done before kc
    _close(a[fin & before], b[fin & before], 1e-6, 1e-9, f"{where}: delta_min")
    _close(a[fin & ~before], b[fin & ~before], 1e-2, 1e-3, f"{where}: delta_min")


@pytest.mark.parametrize("seed", [1000, 1001, 1002])
def test_trace_equals_oracle_points64_fp64(seed):
    p = W.small_points_problem(seed)
    say(f"{p.name} fp64 traced solve")
    C = dvec(p.C)
    f, g, st, tg, _ = eot.eot_solve_ex(C, dvec(p.r), dvec(p.c), trace=True,
                                       **_opts(p, precision="fp64"))
    u, v, ost, to, _ = O.solve_ex(p.C, p.r, p.c, **_opts(p))
    assert st["status"] == 0 and ost["status"] == 0
    say(f"  steps {tg['n_steps']} newton {tg['n_newton']} cg {st['cg_iters']}")
    compare_traces(tg, to, p.name)
    assert st["forcing_misses"] == ost["forcing_misses"]


@pytest.mark.parametrize("kind", ["sqeuclid", "l1"])
def test_trace_equals_oracle_grid784_fp64(kind):
    """28 x 28 grid, both costs (the L1 instance takes the discount-cap /
    forcing-miss path of NewtonSolve at high inverse temperatures)."""
    p = W.mnist_like_problem(2000, kind)
    say(f"{p.name} fp64 traced solve")
    C = torch.from_numpy(p.C).to(DEV)
    f, g, st, tg, _ = eot.eot_solve_ex(C, dvec(p.r), dvec(p.c), trace=True,
                                       **_opts(p, precision="fp64"))
    u, v, ost, to, _ = O.solve_ex(p.C, p.r, p.c, **_opts(p))
    assert st["status"] == 0 and ost["status"] == 0
    say(f"  steps {tg['n_steps']} newton {tg['n_newton']} cg {st['cg_iters']} "
        f"misses {st['forcing_misses']} | oracle misses {ost['forcing_misses']}")
    compare_traces(tg, to, p.name)
    assert st["forcing_misses"] == ost["forcing_misses"]
    assert abs(st["cost"] - ost["cost"]) <= 1e-10 * abs(ost["cost"])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_resume_is_bitwise_the_uninterrupted_solve(prec):
    p = W.small_points_problem(1001)
    C = torch.from_numpy(p.C.astype(np.float32)).to(DEV)      # FP32: both precisions
    r, c = dvec(p.r), dvec(p.c)
    f0, g0, st0, _, _ = eot.eot_solve_ex(C, r, c, **_opts(p, precision=prec))
    for k in (1, 3, 5):
        say(f"{prec}: stop after {k} temperatures, resume")
        fa, ga, sta, _, state = eot.eot_solve_ex(C, r, c, want_state=True,
                                                 allow_not_converged=True,
                                                 **_opts(p, precision=prec, max_mdot=k))
        assert sta["status"] == eot.EOT_ERR_NOT_CONVERGED and state["t"] == k + 1
        f1, g1, st1, _, _ = eot.eot_solve_ex(C, r, c, resume=state, **_opts(p, precision=prec))
        assert st1["status"] == 0
        assert torch.equal(f1, f0) and torch.equal(g1, g0)
        assert st1["mdot_steps"] == st0["mdot_steps"]
        assert sta["newton_steps"] + st1["newton_steps"] == st0["newton_steps"]


def test_saved_state_equals_oracle_state():
    p = W.small_points_problem(1002)
    k = 4
    _, _, sta, _, gs = eot.eot_solve_ex(dvec(p.C), dvec(p.r), dvec(p.c), want_state=True,
                                        allow_not_converged=True,
                                        **_opts(p, precision="fp64", max_mdot=k))
    _, _, ost, _, os_ = O.solve_ex(p.C, p.r, p.c, **_opts(p, max_mdot=k))
    assert ost["status"] == 4 and sta["status"] == eot.EOT_ERR_NOT_CONVERGED
    for key in ("t", "beta", "beta_prev", "q", "rho0"):
        assert gs[key] == os_[key], (key, gs[key], os_[key])
    for key in ("u", "v", "u_prev", "v_prev"):
        a, b = host(gs[key]), os_[key]
        assert np.abs(a - b).max() <= 1e-10 * max(1.0, np.abs(b).max()), key


def test_warm_start_equals_oracle():
    """Warm start from the solution of a nearby problem (other marginals,
    same cost), expressed in cost units at the first temperature."""
    p = W.small_points_problem(1000)
    q = W.small_points_problem(1001)
    uq, vq, _ = O.solve(p.C, q.r, q.c, gamma_init=p.gamma_init, gamma_final=p.gamma_init,
                        tol=1e-6)
    f0, g0 = uq * p.gamma_init, vq * p.gamma_init
    u0, v0 = f0 / p.gamma_init, g0 / p.gamma_init     # the division the library makes
    f, g, st, tg, _ = eot.eot_solve_ex(dvec(p.C), dvec(p.r), dvec(p.c), warm=(dvec(f0), dvec(g0)),
                                       trace=True, **_opts(p, precision="fp64"))
    u, v, ost, to, _ = O.solve_ex(p.C, p.r, p.c, warm=(u0, v0), **_opts(p))
    assert st["status"] == 0 and ost["status"] == 0
    compare_traces(tg, to, "warm")
    assert abs(st["cost"] - ost["cost"]) <= 1e-10 * abs(ost["cost"])
