"""GPU parity of the on-the-fly point-cloud cost (C_ij = |x_i - y_j|^2 / s,
recomputed inside every pass, Sec. 4.2) against the FP64 oracle run on the
dense cost that the oracle builds from the same FP32 points.

Tolerances. FP64 mode: the kernel forms (beta / s) |x - y|^2 in FP64 from
exact differences of FP32 inputs, the oracle beta (|x - y|^2 / s); the two
differ by a few ulp of beta C, i.e. < 1e-13 in a log-marginal for beta <= 1e3,
so 1e-12 is used. Mixed mode: the squared distance is formed in FP32
(|x - y|^2 carries at most ~5 * 2^-24 relative error: the rounded difference
squared, three rounded fused multiply-adds), so each exponent carries an extra
3e-7 beta C_ij on top of the 4e-6 of the FP32 exponent with an exact FP32
cost; the bound used is 4e-6 + 3e-7 beta max C.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2504_02067_amd import eot
from paper_2504_02067_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(msg):
    print(f"[gpu-points] {msg}", flush=True)


def dvec(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def cloud(n, m, d, seed):
    rng = np.random.default_rng(seed)
    X = W.gmm_points(rng, n, d=d)
    Y = W.gmm_points(rng, m, d=d)
    s = W.bbox_scale(X, Y)
    pc = eot.PointCloud(torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV), s)
    return X, Y, s, pc, rng


def mixed_tol(beta, Cmax=1.0):
    return 4e-6 + 3e-7 * beta * Cmax


SHAPES = [(1000, 1500, 3), (300, 4500, 2), (130, 2049, 3), (1, 5, 3), (7, 1, 2), (257, 256, 2)]


@pytest.mark.parametrize("n,m,d", SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_points_marginals_parity(n, m, d, prec):
    gamma = 0.02
    beta = 1.0 / gamma
    X, Y, s, pc, rng = cloud(n, m, d, 100 + n + m + d)
    C = O.sqeuclid_points_cost(X, Y, s)
    r = rng.dirichlet(np.ones(n)); c = rng.dirichlet(np.ones(m))
    u = np.log(r) + rng.standard_normal(n)
    v = np.log(c) - O.log_col_marginal(C, beta, u, np.zeros(m))
    say(f"points marginals n={n} m={m} d={d} {prec}")
    out = eot.eot_marginals(pc, gamma, dvec(u * gamma), dvec(v * gamma), c_for_s=dvec(c),
                            precision=prec)
    torch.cuda.synchronize()
    u, v = O.to_log_units(u * gamma, v * gamma, gamma)
    tol = 1e-12 if prec == "fp64" else mixed_tol(beta, C.max())
    np.testing.assert_allclose(host(out["log_rP"]), O.log_row_marginal(C, beta, u, v), atol=tol, rtol=0)
    np.testing.assert_allclose(host(out["log_cP"]), O.log_col_marginal(C, beta, u, v), atol=tol, rtol=0)
    np.testing.assert_allclose(host(out["s"]), O.row_square_sum(C, beta, u, v, c), rtol=3 * tol, atol=0)
    mref = O.mass(C, beta, u, v)
    assert abs(host(out["mass"])[0] - mref) <= tol * mref


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("rho", [1.0, 0.5])
def test_points_hvp_parity(prec, rho):
    n, m, d, gamma = 700, 2100, 3, 0.05
    beta = 1.0 / gamma
    X, Y, s, pc, rng = cloud(n, m, d, 7)
    C = O.sqeuclid_points_cost(X, Y, s)
    u = -np.log(n) + rng.standard_normal(n)
    v = -np.log(m) - O.log_col_marginal(C, beta, u, np.zeros(m))
    f, g = u * gamma, v * gamma
    u, v = O.to_log_units(f, g, gamma)
    x = rng.standard_normal(n); y = rng.standard_normal(m)
    say(f"points hvp {prec} rho={rho}")
    Hx, Hy = eot.eot_hvp(pc, gamma, dvec(f), dvec(g), rho, dvec(x), dvec(y), precision=prec)
    torch.cuda.synchronize()
    Hx_ref, Hy_ref = O.hvp(C, beta, u, v, rho, x, y)
    ax, ay = O.hvp(C, beta, u, v, rho, np.abs(x), np.abs(y))
    tol = 1e-12 if prec == "fp64" else mixed_tol(beta, C.max())
    assert np.all(np.abs(host(Hx) - Hx_ref) <= tol * ax + 1e-300)
    assert np.all(np.abs(host(Hy) - Hy_ref) <= tol * ay + 1e-300)


def test_points_newton_cg_parity_fp64():
    n, m, d, gamma, eta = 400, 600, 2, 0.05, 0.05
    beta = 1.0 / gamma
    X, Y, s, pc, rng = cloud(n, m, d, 9)
    C = O.sqeuclid_points_cost(X, Y, s)
    r = rng.dirichlet(np.ones(n)) + 1e-3; r /= r.sum()
    c = rng.dirichlet(np.ones(m)) + 1e-3; c /= c.sum()
    u = np.log(r) + 0.5 * rng.standard_normal(n)
    v = np.log(c) - O.log_col_marginal(C, beta, u, np.zeros(m))
    f, g = u * gamma, v * gamma
    u, v = O.to_log_units(f, g, gamma)
    lr = O.log_row_marginal(C, beta, u, v)
    R = O.newton_solve(C, beta, u, v, r, c, lr, eta, 0.0)
    say("points newton_cg fp64")
    out = eot.eot_newton_cg(pc, gamma, dvec(f), dvec(g), dvec(r), dvec(c), eta, 0.0,
                            precision="fp64")
    assert out.levels == R.levels and out.rho_out == R.rho
    scale = np.abs(R.du).max()
    np.testing.assert_allclose(host(out.dir_f) / gamma, R.du, rtol=0, atol=1e-9 * scale)
    np.testing.assert_allclose(host(out.dir_g) / gamma, R.dv, rtol=0, atol=1e-9 * scale)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_points_solve_parity(d, prec):
    p = W.point_cloud_problem(n=512, m=700, d=d, seed=5100 + d)
    p.gamma_final, p.tol = 1e-3, 1e-7
    C = O.sqeuclid_points_cost(p.X, p.Y, p.scale)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    say(f"points solve {p.name} {prec}")
    f, g, st = eot.eot_solve(pc, dvec(p.r), dvec(p.c), gamma_init=p.gamma_init,
                             gamma_final=p.gamma_final, tol=p.tol, precision=prec)
    u, v, ost = O.solve(C, p.r, p.c, gamma_init=p.gamma_init, gamma_final=p.gamma_final,
                        tol=p.tol)
    say(f"  gpu cost={st['cost']:.12e} err={st['err_r'] + st['err_c']:.2e} "
        f"newton={st['newton_steps']} | oracle cost={ost['cost']:.12e} newton={ost['newton_steps']}")
    assert st["status"] == 0 and ost["status"] == 0
    assert st["err_r"] + st["err_c"] <= p.tol
    rel = abs(st["cost"] - ost["cost"]) / ost["cost"]
    assert rel <= (1e-10 if prec == "fp64" else 1e-5)
    # the oracle re-evaluates the GPU potentials on the dense cost
    gu, gv = O.to_log_units(host(f), host(g), p.gamma_final)
    beta = 1.0 / p.gamma_final
    er = np.abs(np.exp(O.log_row_marginal(C, beta, gu, gv)) - p.r).sum()
    ec = np.abs(np.exp(O.log_col_marginal(C, beta, gu, gv)) - p.c).sum()
    assert er + ec <= 2 * p.tol
    if prec == "fp64":
        assert st["mdot_steps"] == ost["mdot_steps"] and st["newton_steps"] == ost["newton_steps"]


def test_points_match_dense_grid_cost():
    """Integer grid positions as points give the dense grid cost exactly, so the
    two cost kinds must agree to FP64 rounding (the grid problem of a batch)."""
    p = W.batch_problem(3)
    side = int(round(np.sqrt(p.n)))
    gamma = p.gamma_final
    Cd = torch.from_numpy(W.grid_cost(side, "sqeuclid", np.float64)).to(DEV)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    rng = np.random.default_rng(2)
    f = gamma * (np.log(p.r) + rng.standard_normal(p.n))
    g = gamma * (np.log(p.c) + rng.standard_normal(p.m))
    say(f"points vs dense grid side={side}")
    a = eot.eot_marginals(pc, gamma, dvec(f), dvec(g), precision="fp64")
    b = eot.eot_marginals(Cd, gamma, dvec(f), dvec(g), precision="fp64")
    np.testing.assert_allclose(host(a["log_rP"]), host(b["log_rP"]), atol=1e-12, rtol=0)
    np.testing.assert_allclose(host(a["log_cP"]), host(b["log_cP"]), atol=1e-12, rtol=0)


@pytest.mark.slow
def test_points_full_size_sampled_marginals():
    """n = m = 2^20 Gaussian-mixture clouds in R^3 (the full point-cloud
    workload: partial buffers would not fit, so the pass accumulates its
    outputs atomically): 32 sampled rows and columns recomputed by the oracle,
    and the mass identity sum r(P) = sum c(P)."""
    p = W.point_cloud_problem()
    n = p.n
    gamma = 1e-2
    beta = 1.0 / gamma
    rng = np.random.default_rng(1)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    u = np.log(p.r) + 0.5 * rng.standard_normal(n)
    v = np.log(p.c) + 0.5 * rng.standard_normal(n)
    f, g = u * gamma, v * gamma
    u, v = O.to_log_units(f, g, gamma)
    rows = np.sort(rng.choice(n, 32, replace=False))
    cols = np.sort(rng.choice(n, 32, replace=False))
    lr_ref = O.log_row_marginal(O.sqeuclid_points_cost(p.X[rows], p.Y, p.scale), beta, u[rows], v)
    lc_ref = O.log_col_marginal(O.sqeuclid_points_cost(p.X, p.Y[cols], p.scale), beta, u, v[cols])
    for prec, tol in (("mixed", mixed_tol(beta)), ("fp64", 1e-12)):
        say(f"points full-size 2^20 marginals {prec}")
        out = eot.eot_marginals(pc, gamma, dvec(f), dvec(g), precision=prec,
                                want=("log_rP", "log_cP"))
        torch.cuda.synchronize()
        lr, lc = host(out["log_rP"]), host(out["log_cP"])
        np.testing.assert_allclose(lr[rows], lr_ref, atol=tol, rtol=0)
        np.testing.assert_allclose(lc[cols], lc_ref, atol=tol, rtol=0)
        m1 = np.exp(lr).sum(); m2 = np.exp(lc).sum()
        assert abs(m1 - m2) <= 10 * tol * m1


def test_points_full_size_sampled_hvp():
    """The point-cloud HVP the benchmark times (n = m = 2^20 in R^3, row shift
    from the marginals, rho = 1, mixed): Hx on 24 sampled rows and Hy on 24
    sampled columns recomputed by the oracle from the points."""
    p = W.point_cloud_problem()
    n = p.n
    gamma, rho = 1e-2, 1.0
    beta = 1.0 / gamma
    rng = np.random.default_rng(2)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    u = np.log(p.r) + 0.5 * rng.standard_normal(n)
    v = np.log(p.c) + 0.5 * rng.standard_normal(n)
    f, g = u * gamma, v * gamma
    u, v = O.to_log_units(f, g, gamma)
    x = rng.standard_normal(n); y = rng.standard_normal(n)
    rows = np.sort(rng.choice(n, 24, replace=False))
    cols = np.sort(rng.choice(n, 24, replace=False))
    Crows = O.sqeuclid_points_cost(p.X[rows], p.Y, p.scale)
    Ccols = O.sqeuclid_points_cost(p.X, p.Y[cols], p.scale)
    hx_ref, _ = O.hvp(Crows, beta, u[rows], v, rho, x[rows], y)
    ax, _ = O.hvp(Crows, beta, u[rows], v, rho, np.abs(x[rows]), np.abs(y))
    _, hy_ref = O.hvp(Ccols, beta, u, v[cols], rho, x, y[cols])
    _, ay = O.hvp(Ccols, beta, u, v[cols], rho, np.abs(x), np.abs(y[cols]))
    say("points full-size 2^20 hvp mixed")
    fd, gd = dvec(f), dvec(g)
    shift = eot.eot_marginals(pc, gamma, fd, gd, precision="mixed", want=("log_rP",))["log_rP"]
    Hx, Hy = eot.eot_hvp(pc, gamma, fd, gd, rho, dvec(x), dvec(y), row_shift=shift,
                         precision="mixed")
    torch.cuda.synchronize()
    tol = mixed_tol(beta, max(Crows.max(), Ccols.max()))
    assert np.all(np.abs(host(Hx)[rows] - hx_ref) <= tol * ax + 1e-300)
    assert np.all(np.abs(host(Hy)[cols] - hy_ref) <= tol * ay + 1e-300)
    # the same product with the diagonal blocks from the library's mixed marginals
    say("points full-size 2^20 hvp with marginals, mixed")
    mg = eot.eot_marginals(pc, gamma, fd, gd, row_shift=shift, precision="mixed",
                           want=("log_rP", "log_cP"))
    Hx, Hy = eot.eot_hvp_with_marginals(pc, gamma, fd, gd, mg["log_rP"], mg["log_cP"], rho,
                                        dvec(x), dvec(y), precision="mixed")
    torch.cuda.synchronize()
    assert np.all(np.abs(host(Hx)[rows] - hx_ref) <= tol * ax + 1e-300)
    assert np.all(np.abs(host(Hy)[cols] - hy_ref) <= tol * ay + 1e-300)


@pytest.mark.parametrize("d,n,m", [(3, 20000, 17000), (2, 16384, 16500)])
def test_points_row_pass_rows_on_lanes(d, n, m):
    """Mixed row sums of large clouds go through the rows-on-lanes kernel
    (k_rows_pts: at least 512 workgroups of 256 rows x 2048 columns): log r(P)
    (rows only) on 48 sampled rows against the oracle and every row against the
    library's FP64 pass. (Its weighted form carries the CG of the large solves
    in tests/test_gpu_configs.py.)"""
    gamma = 0.02
    beta = 1.0 / gamma
    X, Y, s, pc, rng = cloud(n, m, d, 500 + d)
    u = -np.log(n) + rng.standard_normal(n)
    v = -np.log(m) + rng.standard_normal(m)
    f, g = u * gamma, v * gamma
    u, v = O.to_log_units(f, g, gamma)
    rows = np.sort(rng.choice(n, 48, replace=False))
    Crows = O.sqeuclid_points_cost(X[rows], Y, s)
    lr_ref = O.log_row_marginal(Crows, beta, u[rows], v)
    tol = mixed_tol(beta, Crows.max())
    say(f"points rows-on-lanes row pass d={d} {n}x{m}")
    fd, gd = dvec(f), dvec(g)
    lr64 = host(eot.eot_marginals(pc, gamma, fd, gd, precision="fp64", want=("log_rP",))["log_rP"])
    lr32 = host(eot.eot_marginals(pc, gamma, fd, gd, precision="mixed", want=("log_rP",))["log_rP"])
    torch.cuda.synchronize()
    assert np.abs(lr64[rows] - lr_ref).max() <= 1e-12
    assert np.abs(lr32[rows] - lr_ref).max() <= tol
    assert np.abs(lr32 - lr64).max() <= tol


def test_points_gradient_mixed_large_keeps_exact_row_sums():
    """The gradient's CG on a large cloud (n = m = 16384, d = 2: the row pass is
    the rows-on-lanes kernel) runs its row sums in FP64 per entry: the mixed CG
    takes about as many iterations as the FP64 one and reaches the same
    gradient to the mixed tolerance."""
    n = 16384
    p = W.point_cloud_problem(n=n, m=n, d=2, seed=71)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    gamma = 0.01
    f, g, st = eot.eot_solve(pc, dvec(p.r), dvec(p.c), gamma_init=1.0 / 8.0, gamma_final=gamma,
                             tol=1e-7, precision="mixed")
    say("points 16384 gradient, FP64 and mixed CG")
    a = eot.eot_gradient(pc, gamma, f, g, w_W=0.5, w_S=1.0, tol=1e-8)
    b = eot.eot_gradient(pc, gamma, f, g, w_W=0.5, w_S=1.0, tol=1e-8, precision="mixed")
    torch.cuda.synchronize()
    say(f"  CG iterations fp64 {a['cg_iters']}, mixed {b['cg_iters']}")
    assert b["cg_iters"] <= 1.5 * a["cg_iters"] + 10
    for name in ("X", "Y", "r"):
        x, y = host(a[name]), host(b[name])
        assert np.abs(x - y).max() <= 1e-4 * np.abs(x).max(), name
