"""GPU against the oracle on the configurations the kernel-level tests do not
reach: the 28 x 28 grid with the L1 cost in mixed precision, the 16384 x 16384
grid at its final temperature 1e-5 (inverse temperature 1e5) in the state the
benchmark's solve leaves, the 3-D Gaussian-mixture clouds solved down to their
final temperature 1e-4 (n = m = 4096 against a stored oracle solve, and
sampled rows / columns of the 65536-point twin at the solve's potentials), and
the ablation switches of Sec. 3.3 (fixed q), App. B (rho_0 = 0) and Sec. 3.4
(w_r) step by step against the oracle with the same switches.

Each sampled check prints the measured error beside its bound."""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_2504_02067_amd import eot
from paper_2504_02067_amd import workloads as W

from test_gpu_trace import compare_traces

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(msg):
    print(f"[gpu-configs] {msg}", flush=True)


def dvec(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def test_grid784_l1_mixed_cost():
    p = W.mnist_like_problem(2000, "l1")
    C = torch.from_numpy(p.C).to(DEV)
    f, g, st = eot.eot_solve(C, dvec(p.r), dvec(p.c), gamma_init=p.gamma_init,
                             gamma_final=p.gamma_final, tol=p.tol, precision="mixed")
    u, v, ost = O.solve(p.C, p.r, p.c, gamma_init=p.gamma_init, gamma_final=p.gamma_final,
                        tol=p.tol)
    rel = abs(st["cost"] - ost["cost"]) / ost["cost"]
    say(f"grid28 l1 mixed: cost rel diff {rel:.2e}, err {st['err_r'] + st['err_c']:.2e}, "
        f"stalls {st['mixed_stalls']}, range retries {st['range_retries']}")
    assert st["status"] == 0 and ost["status"] == 0
    assert st["err_r"] + st["err_c"] <= p.tol
    assert rel <= 1e-5


def test_grid16384_final_temperature_sampled():
    """The benchmark's solve (mixed, temperature 1/32 -> 1e-5): at its output
    potentials, 48 sampled rows and columns of log r(P), log c(P) and of the
    HVP (rho = 1) in both precisions against the oracle on those rows and
    columns of the cost."""
    side = 128
    n = side * side
    p = W.large_grid_problem(3000)
    C = W.grid_cost_device(side, "sqeuclid", DEV)
    say("grid128 mixed solve to 1e-5")
    f, g, st = eot.eot_solve(C, dvec(p.r), dvec(p.c), gamma_init=p.gamma_init,
                             gamma_final=p.gamma_final, tol=p.tol, precision="mixed")
    assert st["status"] == 0 and st["err_r"] + st["err_c"] <= p.tol
    gamma = p.gamma_final
    beta = 1.0 / gamma
    fh, gh = host(f), host(g)
    u, v = O.to_log_units(fh, gh, gamma)
    rng = np.random.default_rng(16384)
    rows = np.sort(rng.choice(n, 48, replace=False))
    cols = np.sort(rng.choice(n, 48, replace=False))
    Crows = W.grid_cost_rows(side, rows)
    Ccols = W.grid_cost_rows(side, cols).T.copy()          # symmetric grid cost
    lr_ref = O.log_row_marginal(Crows, beta, u[rows], v)
    lc_ref = O.log_col_marginal(Ccols, beta, u, v[cols])
    x = rng.standard_normal(n); y = rng.standard_normal(n)
    hx_ref, _ = O.hvp(Crows, beta, u[rows], v, 1.0, x[rows], y)
    ax, _ = O.hvp(Crows, beta, u[rows], v, 1.0, np.abs(x[rows]), np.abs(y))
    _, hy_ref = O.hvp(Ccols, beta, u, v[cols], 1.0, x, y[cols])
    _, ay = O.hvp(Ccols, beta, u, v[cols], 1.0, np.abs(x), np.abs(y[cols]))
    # FP64: each side rounds the exponent u + v - beta C once at |beta C| up to 1e5,
    # 2^-52 * 1e5 = 2.2e-11 apart at most; mixed: the FP32 exponent's 4e-6
    tol64 = 1e-12 + 2.0 ** -52 * beta * float(Crows.max())
    for prec, tol in (("fp64", tol64), ("mixed", 4e-6)):
        out = eot.eot_marginals(C, gamma, f, g, precision=prec, want=("log_rP", "log_cP"))
        Hx, Hy = eot.eot_hvp(C, gamma, f, g, 1.0, dvec(x), dvec(y), row_shift=out["log_rP"],
                             precision=prec)
        torch.cuda.synchronize()
        er = np.abs(host(out["log_rP"])[rows] - lr_ref).max()
        ec = np.abs(host(out["log_cP"])[cols] - lc_ref).max()
        ex = (np.abs(host(Hx)[rows] - hx_ref) / ax).max()
        ey = (np.abs(host(Hy)[cols] - hy_ref) / ay).max()
        say(f"grid128 at beta 1e5, {prec}: log r(P) {er:.2e}, log c(P) {ec:.2e}, "
            f"Hx {ex:.2e}, Hy {ey:.2e} (bound {tol:.1e})")
        assert max(er, ec, ex, ey) <= tol
    del C
    torch.cuda.empty_cache()


def _cloud(n):
    p = W.point_cloud_problem(n=n, seed=5000)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    return p, pc


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_gmm3d_4096_solve_against_stored_oracle(prec):
    """The full solve of the n = m = 4096 twin of the 3-D point-cloud workload
    (temperature 1/32 -> 1e-4, tol 1e-4) on the on-the-fly cost, against the
    oracle's dense solve stored by tests/golden/make_oracle_goldens.py."""
    ref = json.load(open(os.path.join(GOLDEN, "gmm3d_n4096_oracle.json")))
    p, pc = _cloud(4096)
    assert p.name == ref["problem"]
    f, g, st = eot.eot_solve(pc, dvec(p.r), dvec(p.c), gamma_init=p.gamma_init,
                             gamma_final=p.gamma_final, tol=p.tol, precision=prec)
    rel = abs(st["cost"] - ref["cost"]) / ref["cost"]
    say(f"gmm3d 4096 {prec}: cost rel diff {rel:.2e}, newton {st['newton_steps']} "
        f"(oracle {ref['newton_steps']}), mdot {st['mdot_steps']} ({ref['mdot_steps']}), "
        f"err {st['err_r'] + st['err_c']:.2e}")
    assert st["status"] == 0 and ref["status"] == 0
    assert st["err_r"] + st["err_c"] <= p.tol
    if prec == "fp64":
        assert rel <= 1e-10
        assert st["mdot_steps"] == ref["mdot_steps"]
        assert st["newton_steps"] == ref["newton_steps"]
    else:
        assert rel <= 1e-5


def test_gmm3d_65536_final_temperature_sampled():
    """The n = m = 65536 twin solved in mixed precision to 1e-4; at its output
    potentials (inverse temperature 1e4 / scale), 32 sampled rows and columns
    of the marginals in both precisions against the oracle on the dense rows
    and columns of the cost (rows also from a rows-only pass). Mixed bound: 4e-6
    from the FP32 exponent plus 3e-7 beta max C from the FP32 |x - y|^2."""
    p, pc = _cloud(65536)
    say("gmm3d 65536 mixed solve to 1e-4")
    f, g, st = eot.eot_solve(pc, dvec(p.r), dvec(p.c), gamma_init=p.gamma_init,
                             gamma_final=p.gamma_final, tol=p.tol, precision="mixed")
    assert st["status"] == 0 and st["err_r"] + st["err_c"] <= p.tol
    gamma = p.gamma_final
    beta = 1.0 / gamma
    u, v = O.to_log_units(host(f), host(g), gamma)
    rng = np.random.default_rng(65536)
    rows = np.sort(rng.choice(p.n, 32, replace=False))
    cols = np.sort(rng.choice(p.m, 32, replace=False))
    Crows = O.sqeuclid_points_cost(p.X[rows], p.Y, p.scale)
    Ccols = O.sqeuclid_points_cost(p.X, p.Y[cols], p.scale)
    lr_ref = O.log_row_marginal(Crows, beta, u[rows], v)
    lc_ref = O.log_col_marginal(Ccols, beta, u, v[cols])
    cmax = max(Crows.max(), Ccols.max())
    for prec, tol in (("fp64", 1e-12), ("mixed", 4e-6 + 3e-7 * beta * cmax)):
        out = eot.eot_marginals(pc, gamma, f, g, precision=prec, want=("log_rP", "log_cP"))
        torch.cuda.synchronize()
        er = np.abs(host(out["log_rP"])[rows] - lr_ref).max()
        ec = np.abs(host(out["log_cP"])[cols] - lc_ref).max()
        say(f"gmm3d 65536 at beta {beta:.0e}, {prec}: log r(P) {er:.2e}, log c(P) {ec:.2e} "
            f"(bound {tol:.1e})")
        assert max(er, ec) <= tol
        # rows alone: in mixed precision the rows-on-lanes kernel (k_rows_pts)
        lr = host(eot.eot_marginals(pc, gamma, f, g, precision=prec, want=("log_rP",))["log_rP"])
        torch.cuda.synchronize()
        assert np.abs(lr[rows] - lr_ref).max() <= tol


SWITCHES = [dict(adaptive_q=0, q1=2.0), dict(adaptive_q=0, q1=4.0), dict(adaptive_rho0=0),
            dict(w_r=0.25), dict(w_r=0.35)]


@pytest.mark.parametrize("sw", SWITCHES, ids=lambda d: ",".join(f"{k}={v}" for k, v in d.items()))
@pytest.mark.parametrize("seed", [1000, 1002])
def test_ablation_switches_step_by_step(sw, seed):
    p = W.small_points_problem(seed)
    kw = dict(gamma_init=p.gamma_init, gamma_final=p.gamma_final, tol=p.tol, **sw)
    f, g, st, tg, _ = eot.eot_solve_ex(dvec(p.C), dvec(p.r), dvec(p.c), trace=True,
                                       precision="fp64", **kw)
    u, v, ost, to, _ = O.solve_ex(p.C, p.r, p.c, **kw)
    say(f"{p.name} {sw}: mdot {st['mdot_steps']} newton {st['newton_steps']} "
        f"cg {st['cg_iters']} (oracle {ost['mdot_steps']}/{ost['newton_steps']}/{ost['cg_iters']})")
    assert st["status"] == 0 and ost["status"] == 0
    compare_traces(tg, to, f"{p.name} {sw}")
    if sw.get("adaptive_q") == 0:                 # geometric schedule at the fixed q
        b = to["beta"]
        assert np.all(b[1:] == np.minimum(b[:-1] * sw["q1"], 1.0 / p.gamma_final))
    if sw.get("adaptive_rho0") == 0:
        assert np.all(tg["rho0"] == 0.0)
    assert abs(st["cost"] - ost["cost"]) <= 1e-10 * abs(ost["cost"])
