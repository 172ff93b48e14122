"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Kernel level (marginals, preconditioner sums, Hessian-vector products) on
shapes that span several tiles in both directions with ragged tails, the
degenerate 1-row / 1-column shapes, padded leading dimensions, FP64 and
FP32 costs; NewtonSolve directions; full solves; and, at the 16384 x 16384
size of the throughput benchmark, sampled rows / columns recomputed by the
oracle. Tolerances: FP64 mode 1e-10 relative or tighter; mixed mode as
stated per test (FP32 plan entries, FP64 accumulation).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2504_02067_amd import eot
from paper_2504_02067_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(msg):
    print(f"[gpu-parity] {msg}", flush=True)


def dvec(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def random_case(n, m, seed, gamma, cdtype=np.float32, spread=2.0):
    """Random costs in [0, 1] and potentials whose plan is spread over many
    orders of magnitude (like an iterate of the solver at temperature gamma)."""
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, 1.0, size=(n, m)).astype(cdtype)
    r = rng.dirichlet(np.ones(n)); c = rng.dirichlet(np.ones(m))
    u = np.log(r) + spread * rng.standard_normal(n)
    v = np.log(c) + spread * rng.standard_normal(m)
    f, g = u * gamma, v * gamma            # cost units
    return C, f, g, r, c


def to_log(f, g, gamma):
    return O.to_log_units(f, g, gamma)


SHAPES = [
    (64, 64, np.float64),      # small FP64 problem
    (784, 784, np.float32),    # 28 x 28 grid size
    (300, 4500, np.float32),   # 3 x 3 tiles, ragged both ways
    (130, 2049, np.float32),   # one past a tile in both directions
    (1, 5, np.float32),
    (7, 1, np.float32),
    (1, 1, np.float64),
]


@pytest.mark.parametrize("n,m,cdt", SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("shift", [False, True])
def test_marginals_parity(n, m, cdt, prec, shift):
    gamma = 0.02
    C, f, g, r, c = random_case(n, m, 11 + n + m, gamma, cdt)
    if prec == "mixed" and cdt == np.float64:
        # mixed precision reads an FP32 cost: the library rejects an FP64 one
        with pytest.raises(eot.EotError) as e:
            eot.eot_marginals(torch.from_numpy(C).to(DEV), gamma, dvec(f), dvec(g),
                              precision=prec)
        assert e.value.status == eot.EOT_ERR_UNSUPPORTED
        return
    u, v = to_log(f, g, gamma)
    beta = 1.0 / gamma
    lr_ref = O.log_row_marginal(C, beta, u, v)
    lc_ref = O.log_col_marginal(C, beta, u, v)
    s_ref = O.row_square_sum(C, beta, u, v, c)
    mass_ref = O.mass(C, beta, u, v)
    rs = dvec(lr_ref + np.random.default_rng(1).uniform(-3, 3, n)) if shift else None
    say(f"marginals n={n} m={m} {np.dtype(cdt).name} {prec} shift={shift}")
    out = eot.eot_marginals(torch.from_numpy(C).to(DEV), gamma, dvec(f), dvec(g), row_shift=rs,
                            c_for_s=dvec(c), precision=prec)
    torch.cuda.synchronize()
    # Mixed precision: each plan entry carries ~1.2e-7 + 8.3e-8 |log2(P_ij / max_j P_ij)|
    # relative error (one FP32 rounding of the exponent, v_exp_f32); entries up to
    # 2^-40 below their row maximum still matter to a small column, hence 4e-6 per
    # log-marginal, while mass-weighted (L1) errors stay ~1e-7.
    tol = 1e-12 if prec == "fp64" else 4e-6
    lr, lc = host(out["log_rP"]), host(out["log_cP"])
    np.testing.assert_allclose(lr, lr_ref, rtol=0, atol=tol)
    np.testing.assert_allclose(lc, lc_ref, rtol=0, atol=tol)
    np.testing.assert_allclose(host(out["s"]), s_ref, rtol=3 * tol, atol=0)
    assert abs(host(out["mass"])[0] - mass_ref) <= tol * mass_ref
    wtol = 1e-12 if prec == "fp64" else 3e-7
    assert np.abs(np.exp(lr) - np.exp(lr_ref)).sum() <= wtol * np.exp(lr_ref).sum()
    assert np.abs(np.exp(lc) - np.exp(lc_ref)).sum() <= wtol * np.exp(lc_ref).sum()


def test_marginals_padded_leading_dimension():
    # ldc > m (rows not 16-byte aligned: scalar-load path)
    n, m, gamma = 257, 1030, 0.05
    C, f, g, r, c = random_case(n, m, 5, gamma)
    buf = np.zeros((n, m + 3), dtype=np.float32)
    buf[:, :m] = C
    Cd = torch.from_numpy(buf).to(DEV)[:, :m]
    assert Cd.stride(0) == m + 3
    u, v = to_log(f, g, gamma)
    beta = 1.0 / gamma
    for prec, tol in (("fp64", 1e-12), ("mixed", 4e-6)):
        say(f"padded ldc {prec}")
        out = eot.eot_marginals(Cd, gamma, dvec(f), dvec(g), precision=prec)
        np.testing.assert_allclose(host(out["log_rP"]), O.log_row_marginal(C, beta, u, v), atol=tol, rtol=0)
        np.testing.assert_allclose(host(out["log_cP"]), O.log_col_marginal(C, beta, u, v), atol=tol, rtol=0)


@pytest.mark.parametrize("n,m,ldc", [(257, 1030, 1032), (300, 2052, 2060), (9, 5, 8)])
@pytest.mark.parametrize("pad", [np.nan, -np.inf])
@pytest.mark.parametrize("cdt", [np.float32, np.float64])
def test_padding_is_never_read(n, m, ldc, pad, cdt):
    """Rows padded to a multiple of 4 elements (16-byte aligned rows) with NaN
    or -inf in the padding: marginals and HVPs equal those of the unpadded
    cost (m % 4 != 0 and m % 4 == 0 with ldc > m)."""
    gamma = 0.05
    C, f, g, r, c = random_case(n, m, n + ldc, gamma, cdt)
    buf = np.full((n, ldc), pad, dtype=cdt)
    buf[:, :m] = C
    Cd = torch.from_numpy(buf).to(DEV)[:, :m]
    assert Cd.stride(0) == ldc and Cd.data_ptr() % 16 == 0
    u, v = to_log(f, g, gamma)
    beta = 1.0 / gamma
    rng = np.random.default_rng(n)
    x, y = rng.standard_normal(n), rng.standard_normal(m)
    Hx_ref, Hy_ref = O.hvp(C, beta, u, v, 0.5625, x, y)
    ax, ay = O.hvp(C, beta, u, v, 0.5625, np.abs(x), np.abs(y))
    for prec, tol in (("fp64", 1e-12), ("mixed", 4e-6)):
        if prec == "mixed" and cdt == np.float64:
            continue
        say(f"padding {pad} ldc={ldc} m={m} {cdt.__name__} {prec}")
        out = eot.eot_marginals(Cd, gamma, dvec(f), dvec(g), precision=prec)
        np.testing.assert_allclose(host(out["log_rP"]), O.log_row_marginal(C, beta, u, v),
                                   atol=tol, rtol=0)
        np.testing.assert_allclose(host(out["log_cP"]), O.log_col_marginal(C, beta, u, v),
                                   atol=tol, rtol=0)
        Hx, Hy = eot.eot_hvp(Cd, gamma, dvec(f), dvec(g), 0.5625, dvec(x), dvec(y),
                             precision=prec)
        assert (np.abs(host(Hx) - Hx_ref) <= tol * ax).all()
        assert (np.abs(host(Hy) - Hy_ref) <= tol * ay).all()


@pytest.mark.parametrize("n,m,cdt", [(64, 64, np.float64), (300, 4500, np.float32),
                                     (130, 2049, np.float32), (1, 3, np.float32)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("rho", [1.0, 0.5625, 0.0])
def test_hvp_parity(n, m, cdt, prec, rho):
    gamma = 0.05
    C, f, g, r, c = random_case(n, m, 3 * n + m, gamma, cdt, spread=1.0)
    if prec == "mixed" and cdt == np.float64:
        # mixed precision reads an FP32 cost: the library rejects an FP64 one
        with pytest.raises(eot.EotError) as e:
            eot.eot_hvp(torch.from_numpy(C).to(DEV), gamma, dvec(f), dvec(g), rho,
                        dvec(np.ones(n)), dvec(np.ones(m)), precision=prec)
        assert e.value.status == eot.EOT_ERR_UNSUPPORTED
        return
    u, v = to_log(f, g, gamma)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(n); y = rng.standard_normal(m)
    Hx_ref, Hy_ref = O.hvp(C, 1.0 / gamma, u, v, rho, x, y)
    say(f"hvp n={n} m={m} {prec} rho={rho}")
    Hx, Hy = eot.eot_hvp(torch.from_numpy(C).to(DEV), gamma, dvec(f), dvec(g), rho, dvec(x),
                         dvec(y), precision=prec)
    torch.cuda.synchronize()
    # scale: |r(P)| |x| + sqrt(rho) P |y| per row, likewise per column
    ax, ay = O.hvp(C, 1.0 / gamma, u, v, rho, np.abs(x), np.abs(y))
    tol = 1e-12 if prec == "fp64" else 4e-6
    assert np.all(np.abs(host(Hx) - Hx_ref) <= tol * ax + 1e-300)
    assert np.all(np.abs(host(Hy) - Hy_ref) <= tol * ay + 1e-300)


def _fixed_instance(n, m, seed, gamma, cdt=np.float32, spread=0.5):
    """Random instance after the column fix (c(P) = c), as NewtonSolve sees it."""
    rng = np.random.default_rng(seed)
    C = rng.uniform(0, 1, size=(n, m)).astype(cdt)
    r = rng.dirichlet(np.ones(n)) + 1e-3; r /= r.sum()
    c = rng.dirichlet(np.ones(m)) + 1e-3; c /= c.sum()
    beta = 1.0 / gamma
    u = np.log(r) + spread * rng.standard_normal(n)
    v = np.log(c) - O.log_col_marginal(C, beta, u, np.zeros(m))
    return C, r, c, u, v, beta


@pytest.mark.parametrize("n,m,eta,rho0", [(200, 150, 0.3, 0.0), (200, 150, 1e-3, 0.0),
                                          (513, 2100, 0.05, 0.75), (64, 64, 0.01, 0.9375)])
def test_newton_cg_parity_fp64(n, m, eta, rho0):
    gamma = 0.05
    C, r, c, u, v, beta = _fixed_instance(n, m, n + m, gamma)
    lr = O.log_row_marginal(C, beta, u, v)
    R = O.newton_solve(C, beta, u, v, r, c, lr, eta, rho0)
    say(f"newton_cg n={n} m={m} eta={eta} rho0={rho0}")
    out = eot.eot_newton_cg(torch.from_numpy(C).to(DEV), gamma, dvec(u * gamma), dvec(v * gamma),
                            dvec(r), dvec(c), eta, rho0, precision="fp64")
    assert out.levels == R.levels and out.rho_out == R.rho
    assert out.forcing_miss == R.forcing_miss == 0
    du = host(out.dir_f) / gamma
    dv = host(out.dir_g) / gamma
    scale = np.abs(R.du).max()
    np.testing.assert_allclose(du, R.du, rtol=0, atol=1e-9 * scale)
    np.testing.assert_allclose(dv, R.dv, rtol=0, atol=1e-9 * scale)
    # the GPU direction meets the forcing inequality, checked by the oracle
    rP = np.exp(lr)
    e = O.fr_apply(C, beta, u, v, rP, c, 1.0, du) + (rP - r)
    assert np.abs(e).sum() <= eta * np.abs(rP - r).sum() * (1 + 1e-9)


@pytest.mark.parametrize("max_cg", [1, 2, 3])
def test_newton_cg_iteration_cap_fp64(max_cg):
    """CG capped at a few iterations: the paced launches stop at the cap, and
    NewtonSolve's levels, final rho, iteration count, forcing miss and direction
    match the oracle's under the same cap."""
    gamma = 0.05
    C, r, c, u, v, beta = _fixed_instance(200, 150, 5, gamma)
    lr = O.log_row_marginal(C, beta, u, v)
    R = O.newton_solve(C, beta, u, v, r, c, lr, 0.05, 0.0, max_cg=max_cg)
    say(f"newton_cg cap max_cg={max_cg}")
    out = eot.eot_newton_cg(torch.from_numpy(C).to(DEV), gamma, dvec(u * gamma), dvec(v * gamma),
                            dvec(r), dvec(c), 0.05, 0.0, max_cg=max_cg, precision="fp64")
    assert (out.levels, out.rho_out, out.forcing_miss) == (R.levels, R.rho, R.forcing_miss)
    assert out.cg_iters == R.cg_iters
    scale = np.abs(R.du).max()
    np.testing.assert_allclose(host(out.dir_f) / gamma, R.du, rtol=0, atol=1e-9 * scale)
    np.testing.assert_allclose(host(out.dir_g) / gamma, R.dv, rtol=0, atol=1e-9 * scale)


def test_newton_cg_mixed_meets_forcing():
    gamma = 0.02
    C, r, c, u, v, beta = _fixed_instance(700, 900, 21, gamma)
    lr = O.log_row_marginal(C, beta, u, v)
    eta = 0.1
    say("newton_cg mixed 700x900")
    out = eot.eot_newton_cg(torch.from_numpy(C).to(DEV), gamma, dvec(u * gamma), dvec(v * gamma),
                            dvec(r), dvec(c), eta, 0.0, precision="mixed")
    du = host(out.dir_f) / gamma
    rP = np.exp(lr)
    e = O.fr_apply(C, beta, u, v, rP, c, 1.0, du) + (rP - r)
    assert np.abs(e).sum() <= eta * np.abs(rP - r).sum() * 1.01
    R = O.newton_solve(C, beta, u, v, r, c, lr, eta, 0.0)
    rel = np.abs(du - R.du).max() / np.abs(R.du).max()
    say(f"  mixed vs fp64 direction rel diff {rel:.2e}")
    assert rel < 0.2


def _solve_both(p, prec):
    C = torch.from_numpy(p.C).to(DEV)
    f, g, st = eot.eot_solve(C, dvec(p.r), dvec(p.c), gamma_init=p.gamma_init,
                             gamma_final=p.gamma_final, tol=p.tol, precision=prec)
    u, v, ost = O.solve(p.C, p.r, p.c, gamma_init=p.gamma_init, gamma_final=p.gamma_final,
                        tol=p.tol)
    return f, g, st, u, v, ost


@pytest.mark.parametrize("seed", [1000, 1001, 1002])
def test_solve_parity_small_fp64(seed):
    p = W.small_points_problem(seed)
    say(f"solve {p.name} fp64 tol={p.tol}")
    f, g, st, u, v, ost = _solve_both(p, "fp64")
    assert st["status"] == 0 and ost["status"] == 0
    assert st["err_r"] + st["err_c"] <= p.tol
    assert abs(st["cost"] - ost["cost"]) <= 1e-10 * abs(ost["cost"])
    assert abs(st["dual_value"] - p.gamma_final * -ost["dual_value"]) <= 1e-10 * abs(st["dual_value"])
    # the oracle re-evaluates the GPU potentials
    beta = 1.0 / p.gamma_final
    gu, gv = host(f) / p.gamma_final, host(g) / p.gamma_final
    er = np.abs(np.exp(O.log_row_marginal(p.C, beta, gu, gv)) - p.r).sum()
    ec = np.abs(np.exp(O.log_col_marginal(p.C, beta, gu, gv)) - p.c).sum()
    assert er + ec <= p.tol
    assert st["mdot_steps"] == ost["mdot_steps"] and st["newton_steps"] == ost["newton_steps"]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_parity_grid784(prec):
    p = W.mnist_like_problem(2000, "sqeuclid")
    say(f"solve {p.name} {prec}")
    f, g, st, u, v, ost = _solve_both(p, prec)
    say(f"  gpu {st['seconds']:.2f}s cost={st['cost']:.12e} err={st['err_r'] + st['err_c']:.2e} "
        f"newton={st['newton_steps']} cg={st['cg_iters']} | oracle cost={ost['cost']:.12e}")
    assert st["status"] == 0 and ost["status"] == 0
    assert st["err_r"] + st["err_c"] <= p.tol
    rel = abs(st["cost"] - ost["cost"]) / ost["cost"]
    assert rel <= (1e-10 if prec == "fp64" else 1e-5)


def test_full_size_sampled_marginals():
    """16384 x 16384 FP32 cost (1 GiB, built on the device): marginals at
    solver-like potentials, 48 sampled rows and columns recomputed by the
    oracle, both precisions, in the launch configuration of the benchmark."""
    side = 128
    n = side * side
    p = W.large_grid_problem(3000)
    gamma = 1e-3
    beta = 1.0 / gamma
    rng = np.random.default_rng(0)
    u = np.log(p.r) + 0.5 * rng.standard_normal(n)
    v = np.log(p.c) + 0.5 * rng.standard_normal(n)
    say("full-size cost build")
    C = W.grid_cost_device(side, "sqeuclid", DEV)
    rows = np.sort(rng.choice(n, 48, replace=False))
    cols = np.sort(rng.choice(n, 48, replace=False))
    Crows = W.grid_cost_rows(side, rows)
    Ccols = W.grid_cost_rows(side, cols).T.copy()        # symmetric grid cost
    assert np.array_equal(host(C[torch.from_numpy(rows).to(DEV)]), Crows)
    lr_ref = O.log_row_marginal(Crows, beta, u[rows], v)
    lc_ref = O.log_col_marginal(Ccols, beta, u, v[cols])
    for prec, tol in (("fp64", 1e-12), ("mixed", 4e-6)):
        say(f"full-size marginals {prec}")
        out = eot.eot_marginals(C, gamma, dvec(u * gamma), dvec(v * gamma), precision=prec)
        torch.cuda.synchronize()
        np.testing.assert_allclose(host(out["log_rP"])[rows], lr_ref, atol=tol, rtol=0)
        np.testing.assert_allclose(host(out["log_cP"])[cols], lc_ref, atol=tol, rtol=0)
        # sum r(P) = sum c(P) at any size
        m1 = np.exp(host(out["log_rP"])).sum(); m2 = np.exp(host(out["log_cP"])).sum()
        assert abs(m1 - m2) <= 10 * tol * m1
    del C
    torch.cuda.empty_cache()


def test_full_size_sampled_hvp():
    """The benchmark's roofline kernel in its launch configuration: the fused HVP
    on the 16384 x 16384 FP32 cost with the row shift from the marginals and
    rho = 1, both precisions; Hx on 40 sampled rows and Hy on 40 sampled columns
    (plus the first and last) recomputed by the oracle from those rows and
    columns of the cost."""
    side = 128
    n = side * side
    p = W.large_grid_problem(3000)
    gamma, rho = 1e-3, 1.0
    beta = 1.0 / gamma
    rng = np.random.default_rng(4)
    u = np.log(p.r) + 0.5 * rng.standard_normal(n)
    v = np.log(p.c) + 0.5 * rng.standard_normal(n)
    x = rng.standard_normal(n); y = rng.standard_normal(n)
    say("full-size hvp: cost build")
    C = W.grid_cost_device(side, "sqeuclid", DEV)
    rows = np.concatenate([[0, n - 1], np.sort(rng.choice(n, 40, replace=False))])
    cols = np.concatenate([[0, n - 1], np.sort(rng.choice(n, 40, replace=False))])
    Crows = W.grid_cost_rows(side, rows)
    Ccols = W.grid_cost_rows(side, cols).T.copy()        # symmetric grid cost
    hx_ref, _ = O.hvp(Crows, beta, u[rows], v, rho, x[rows], y)
    ax, _ = O.hvp(Crows, beta, u[rows], v, rho, np.abs(x[rows]), np.abs(y))
    _, hy_ref = O.hvp(Ccols, beta, u, v[cols], rho, x, y[cols])
    _, ay = O.hvp(Ccols, beta, u, v[cols], rho, np.abs(x), np.abs(y[cols]))
    f, g = dvec(u * gamma), dvec(v * gamma)
    for prec, tol in (("mixed", 4e-6), ("fp64", 1e-12)):
        say(f"full-size hvp {prec}")
        shift = eot.eot_marginals(C, gamma, f, g, want=("log_rP",), precision=prec)["log_rP"]
        Hx, Hy = eot.eot_hvp(C, gamma, f, g, rho, dvec(x), dvec(y), row_shift=shift,
                             precision=prec)
        torch.cuda.synchronize()
        assert np.all(np.abs(host(Hx)[rows] - hx_ref) <= tol * ax + 1e-300)
        assert np.all(np.abs(host(Hy)[cols] - hy_ref) <= tol * ay + 1e-300)
    del C
    torch.cuda.empty_cache()


@pytest.mark.parametrize("seed", [1000, 1001])
def test_sinkhorn_projection_parity_fp64(seed):
    """MDOT with the Sinkhorn projection (the paper's baseline) on the same
    streaming passes, against the oracle's MDOT-Sinkhorn: same number of
    sweeps and temperature steps, cost within 1e-10."""
    p = W.small_points_problem(seed)
    kw = dict(gamma_init=1e-1, gamma_final=1e-2, tol=1e-9)
    say(f"MDOT-Sinkhorn {p.name}")
    C = torch.from_numpy(p.C).to(DEV)
    f, g, st = eot.eot_solve(C, dvec(p.r), dvec(p.c), projection="sinkhorn", **kw)
    u, v, ost = O.solve(p.C, p.r, p.c, projection=1, **kw)
    assert st["status"] == 0 and ost["status"] == 0
    assert st["sinkhorn_iters"] == ost["sinkhorn_iters"] and st["mdot_steps"] == ost["mdot_steps"]
    assert st["newton_steps"] == 0
    assert abs(st["cost"] - ost["cost"]) <= 1e-10 * ost["cost"]


def test_sinkhorn_projection_mixed_grid784():
    p = W.mnist_like_problem(2000, "sqeuclid")
    kw = dict(gamma_init=p.gamma_init, gamma_final=1e-2, tol=1e-6)
    say("MDOT-Sinkhorn grid784 mixed vs fp64")
    C = torch.from_numpy(p.C).to(DEV)
    f, g, st = eot.eot_solve(C, dvec(p.r), dvec(p.c), projection="sinkhorn", precision="mixed", **kw)
    f2, g2, st2 = eot.eot_solve(C, dvec(p.r), dvec(p.c), projection="sinkhorn", **kw)
    say(f"  mixed {st['seconds']:.2f}s sweeps={st['sinkhorn_iters']} | fp64 {st2['seconds']:.2f}s "
        f"sweeps={st2['sinkhorn_iters']}")
    assert st["status"] == 0 and st2["status"] == 0
    assert st["err_r"] + st["err_c"] <= 1e-6
    assert abs(st["cost"] - st2["cost"]) <= 1e-5 * st2["cost"]


@pytest.mark.parametrize("rb", [8, 32, 256])
def test_every_tile_height_gives_the_same_marginals(rb):
    n, m, gamma = 700, 2500, 0.02
    C, f, g, r, c = random_case(n, m, 77, gamma)
    u, v = to_log(f, g, gamma)
    say(f"tile height {rb}")
    eot.eot_set_rows_per_tile(rb)
    try:
        out = eot.eot_marginals(torch.from_numpy(C).to(DEV), gamma, dvec(f), dvec(g), precision="fp64")
        Hx, Hy = eot.eot_hvp(torch.from_numpy(C).to(DEV), gamma, dvec(f), dvec(g), 0.5,
                             dvec(np.ones(n)), dvec(np.ones(m)), precision="mixed")
    finally:
        eot.eot_set_rows_per_tile(0)
    np.testing.assert_allclose(host(out["log_rP"]), O.log_row_marginal(C, 1 / gamma, u, v), atol=1e-12, rtol=0)
    np.testing.assert_allclose(host(out["log_cP"]), O.log_col_marginal(C, 1 / gamma, u, v), atol=1e-12, rtol=0)
    Hx_ref, Hy_ref = O.hvp(C, 1 / gamma, u, v, 0.5, np.ones(n), np.ones(m))
    np.testing.assert_allclose(host(Hx), Hx_ref, rtol=4e-6)
    np.testing.assert_allclose(host(Hy), Hy_ref, rtol=4e-6)
