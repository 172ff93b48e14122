"""GPU parity of the high-dimensional point-cloud passes (d = 16 .. 64, the
x . y contraction on the matrix cores) against the FP64 oracle on the dense
cost it builds from the same FP32 points.

Tolerances. FP64 mode forms |x - y|^2 per entry in FP64: 1e-12, as for d <= 3.
Mixed mode: x . y from BF16 hi/lo parts (three products, FP32 accumulation)
errs by at most ~3 * 2^-17 sum_k |x_k y_k| <= 1.2e-5 (|x|^2 + |y|^2) / 1, and
|x|^2 + |y|^2 - 2 x . y adds ~3 * 2^-24 (|x|^2 + |y|^2); for unit vectors
(|x|^2 + |y|^2 = 2, scale 4) an entry's exponent moves by <= 1.2e-5 beta, so a
log-marginal by at most that plus the 4e-6 of the FP32 exponent.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import gradients as OG
from paper_2504_02067_amd import eot
from paper_2504_02067_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(msg):
    print(f"[gpu-highd] {msg}", flush=True)


def dvec(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def mixed_tol(beta):
    return 4e-6 + 1.2e-5 * beta


def cloud(n, m, d, seed):
    p = W.embedding_problem(n, m, d, seed)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    return p, pc, O.sqeuclid_points_cost(p.X, p.Y, p.scale)


@pytest.mark.parametrize("d", [16, 48, 64])
@pytest.mark.parametrize("n,m", [(300, 700), (129, 513), (1, 40)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_highd_marginals_parity(d, n, m, prec):
    gamma = 0.05
    beta = 1.0 / gamma
    p, pc, C = cloud(n, m, d, 10 * d + n)
    rng = np.random.default_rng(d + m)
    u = np.log(p.r) + rng.standard_normal(n)
    v = np.log(p.c) - O.log_col_marginal(C, beta, u, np.zeros(m))
    f, g = u * gamma, v * gamma
    u, v = O.to_log_units(f, g, gamma)
    say(f"high-d marginals d={d} n={n} m={m} {prec}")
    out = eot.eot_marginals(pc, gamma, dvec(f), dvec(g), c_for_s=dvec(p.c), precision=prec)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == "fp64" else mixed_tol(beta)
    np.testing.assert_allclose(host(out["log_rP"]), O.log_row_marginal(C, beta, u, v), atol=tol, rtol=0)
    np.testing.assert_allclose(host(out["log_cP"]), O.log_col_marginal(C, beta, u, v), atol=tol, rtol=0)
    np.testing.assert_allclose(host(out["s"]), O.row_square_sum(C, beta, u, v, p.c), rtol=3 * tol, atol=0)


@pytest.mark.parametrize("d,n,m", [(16, 130, 517), (32, 400, 600), (48, 257, 129), (64, 333, 1100)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_highd_hvp_parity(d, n, m, prec):
    gamma, rho = 0.05, 0.5
    beta = 1.0 / gamma
    p, pc, C = cloud(n, m, d, 3 + d)
    rng = np.random.default_rng(5)
    u = np.log(p.r) + 0.5 * rng.standard_normal(n)
    v = np.log(p.c) - O.log_col_marginal(C, beta, u, np.zeros(m))
    f, g = u * gamma, v * gamma
    u, v = O.to_log_units(f, g, gamma)
    x = rng.standard_normal(n); y = rng.standard_normal(m)
    say(f"high-d hvp d={d} n={n} m={m} {prec}")
    Hx, Hy = eot.eot_hvp(pc, gamma, dvec(f), dvec(g), rho, dvec(x), dvec(y), precision=prec)
    Hx_ref, Hy_ref = O.hvp(C, beta, u, v, rho, x, y)
    ax, ay = O.hvp(C, beta, u, v, rho, np.abs(x), np.abs(y))
    tol = 1e-12 if prec == "fp64" else mixed_tol(beta)
    assert np.all(np.abs(host(Hx) - Hx_ref) <= tol * ax + 1e-300)
    assert np.all(np.abs(host(Hy) - Hy_ref) <= tol * ay + 1e-300)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_highd_unaligned_points_parity(prec):
    """Y as an element-offset view (4 bytes past a 16-byte boundary): the FP64
    pass and the FP64 row maxima, which read Y in 16-byte vectors, take the
    per-entry kernel instead; marginals (with the row shift) and the HVP against
    the oracle."""
    n, m, d, gamma, rho = 200, 333, 48, 0.05, 0.7
    beta = 1.0 / gamma
    p = W.embedding_problem(n, m, d, 55)
    X = torch.from_numpy(p.X).to(DEV)
    buf = torch.empty(m * d + 1, dtype=torch.float32, device=DEV)
    Y = buf[1:].view(m, d)
    Y.copy_(torch.from_numpy(p.Y))
    assert Y.data_ptr() % 16 == 4
    pc = eot.PointCloud(X, Y, p.scale)
    C = O.sqeuclid_points_cost(p.X, p.Y, p.scale)
    rng = np.random.default_rng(56)
    u = np.log(p.r) + 0.5 * rng.standard_normal(n)
    v = np.log(p.c) + 0.5 * rng.standard_normal(m)
    f, g = u * gamma, v * gamma
    u, v = O.to_log_units(f, g, gamma)
    x = rng.standard_normal(n); y = rng.standard_normal(m)
    say(f"high-d unaligned Y {prec}")
    out = eot.eot_marginals(pc, gamma, dvec(f), dvec(g), precision=prec)
    Hx, Hy = eot.eot_hvp(pc, gamma, dvec(f), dvec(g), rho, dvec(x), dvec(y), precision=prec)
    torch.cuda.synchronize()
    tol = 1e-12 if prec == "fp64" else mixed_tol(beta)
    np.testing.assert_allclose(host(out["log_rP"]), O.log_row_marginal(C, beta, u, v), atol=tol, rtol=0)
    np.testing.assert_allclose(host(out["log_cP"]), O.log_col_marginal(C, beta, u, v), atol=tol, rtol=0)
    Hx_ref, Hy_ref = O.hvp(C, beta, u, v, rho, x, y)
    ax, ay = O.hvp(C, beta, u, v, rho, np.abs(x), np.abs(y))
    assert np.all(np.abs(host(Hx) - Hx_ref) <= tol * ax + 1e-300)
    assert np.all(np.abs(host(Hy) - Hy_ref) <= tol * ay + 1e-300)


@pytest.mark.parametrize("d", [16, 48])
def test_highd_newton_cg_parity_fp64(d):
    """NewtonSolve (Alg. 2) on the matrix-core passes: the same rho levels as the
    oracle and the same direction to CG rounding (the FP64 passes agree with the
    oracle to 1e-12, so the CG iterates track the oracle's)."""
    n, m, gamma, eta = 300, 420, 0.05, 0.05
    beta = 1.0 / gamma
    p, pc, C = cloud(n, m, d, 60 + d)
    rng = np.random.default_rng(61 + d)
    r, c = p.r, p.c
    u = np.log(r) + 0.5 * rng.standard_normal(n)
    v = np.log(c) - O.log_col_marginal(C, beta, u, np.zeros(m))
    f, g = u * gamma, v * gamma
    u, v = O.to_log_units(f, g, gamma)
    lr = O.log_row_marginal(C, beta, u, v)
    R = O.newton_solve(C, beta, u, v, r, c, lr, eta, 0.0)
    say(f"high-d newton_cg d={d} fp64")
    out = eot.eot_newton_cg(pc, gamma, dvec(f), dvec(g), dvec(r), dvec(c), eta, 0.0,
                            precision="fp64")
    assert out.levels == R.levels and out.rho_out == R.rho
    scale = np.abs(R.du).max()
    np.testing.assert_allclose(host(out.dir_f) / gamma, R.du, rtol=0, atol=1e-9 * scale)
    np.testing.assert_allclose(host(out.dir_g) / gamma, R.dv, rtol=0, atol=1e-9 * scale)


def test_highd_newton_cg_mixed_meets_forcing():
    """Mixed CG on the BF16 hi / lo passes: its direction meets the forcing
    inequality of Alg. 2 when checked by the oracle in FP64."""
    n, m, d, gamma, eta = 350, 300, 64, 0.05, 0.1
    beta = 1.0 / gamma
    p, pc, C = cloud(n, m, d, 77)
    rng = np.random.default_rng(78)
    r, c = p.r, p.c
    u = np.log(r) + 0.5 * rng.standard_normal(n)
    v = np.log(c) - O.log_col_marginal(C, beta, u, np.zeros(m))
    f, g = u * gamma, v * gamma
    u, v = O.to_log_units(f, g, gamma)
    lr = O.log_row_marginal(C, beta, u, v)
    say("high-d newton_cg d=64 mixed")
    out = eot.eot_newton_cg(pc, gamma, dvec(f), dvec(g), dvec(r), dvec(c), eta, 0.0,
                            precision="mixed")
    du = host(out.dir_f) / gamma
    rP = np.exp(lr)
    e = O.fr_apply(C, beta, u, v, rP, c, 1.0, du) + (rP - r)
    assert np.abs(e).sum() <= eta * np.abs(rP - r).sum() * 1.01


@pytest.mark.parametrize("d", [16, 32, 48, 64])
def test_highd_gradient_parity(d):
    """eot_gradient on high-dimensional points (FP64 row sums of the cotangent,
    d / 16 lanes per row): dX, dY, dr, dc and S against the oracle's derivative
    formulas on the dense cost built from the same points, at the GPU potentials.
    Tolerance 1e-8 of the largest entry: the S part goes through a CG solve to a
    relative residual of 1e-11."""
    n, m, gamma = 150, 230, 0.05
    p, pc, C = cloud(n, m, d, 90 + d)
    f, g, st = eot.eot_solve(pc, dvec(p.r), dvec(p.c), gamma_init=1.0 / 8.0, gamma_final=gamma,
                             tol=1e-9, precision="fp64")
    assert st["status"] == 0
    say(f"high-d gradient d={d}")
    out = eot.eot_gradient(pc, gamma, f, g, w_W=0.4, w_S=1.1)
    u, v = O.to_log_units(host(f), host(g), gamma)
    G, gr, gc, S, _, _ = OG.vjp(C, 1.0 / gamma, u, v, 0.4, 1.1)
    gX, gY = OG.points_grad(p.X, p.Y, p.scale, G)
    assert abs(out["S"] - S) <= 1e-12 * S
    for key, ref in (("X", gX), ("Y", gY), ("r", gr), ("c", gc)):
        a = host(out[key])
        assert a.shape == ref.shape
        err = np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-300)
        assert err <= 1e-8, (key, err)


def test_highd_autograd_points():
    """The torch.autograd wrapper on d = 32 embeddings: dS/dX and dS/dY from
    backward() against the oracle's formulas at the potentials of the same
    solve (1e-6 of the largest entry: the gradients come back in FP32)."""
    from paper_2504_02067_amd import autograd as AG
    gamma = 0.05
    p, pc, C = cloud(160, 190, 32, 123)
    X = torch.from_numpy(p.X).to(DEV).requires_grad_(True)
    Y = torch.from_numpy(p.Y).to(DEV).requires_grad_(True)
    say("high-d autograd d=32")
    Wv, Sv = AG.entropic_ot_points(X, Y, dvec(p.r), dvec(p.c), gamma, p.scale,
                                   gamma_init=1.0 / 8.0, tol=1e-9)
    Sv.backward()
    assert X.grad.shape == X.shape and Y.grad.shape == Y.shape
    f, g, st = eot.eot_solve(eot.PointCloud(X.detach(), Y.detach(), p.scale), dvec(p.r),
                             dvec(p.c), gamma_init=1.0 / 8.0, gamma_final=gamma, tol=1e-9)
    u, v = O.to_log_units(host(f), host(g), gamma)
    G, *_ = OG.vjp(C, 1.0 / gamma, u, v, 0.0, 1.0)
    gX, gY = OG.points_grad(p.X, p.Y, p.scale, G)
    for a, ref in ((host(X.grad), gX), (host(Y.grad), gY)):
        err = np.abs(a.astype(np.float64) - ref).max() / np.abs(ref).max()
        assert err <= 1e-6, err


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_highd_solve_parity(prec):
    p, pc, C = cloud(300, 400, 64, 11)
    kw = dict(gamma_init=1.0 / 8.0, gamma_final=0.02, tol=1e-6)
    say(f"high-d solve {prec}")
    f, g, st = eot.eot_solve(pc, dvec(p.r), dvec(p.c), precision=prec, **kw)
    u, v, ost = O.solve(C, p.r, p.c, **kw)
    assert st["status"] == 0 and ost["status"] == 0
    assert st["err_r"] + st["err_c"] <= kw["tol"]
    rel = abs(st["cost"] - ost["cost"]) / ost["cost"]
    say(f"  cost rel diff {rel:.2e}")
    assert rel <= (1e-10 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_highd_wide_tiles_sampled(prec):
    """n x m large enough that the pass takes 2048-column tiles (>= 2048 workgroups),
    with a ragged last tile (2500 = 2048 + 452): marginals and the HVP checked on
    sampled rows and columns, each computed by the oracle from its own slice of the
    cost."""
    n, m, d, gamma, rho = 128 * 2048, 2500, 64, 0.05, 0.7
    beta = 1.0 / gamma
    p = W.embedding_problem(n, m, d, 21)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    rng = np.random.default_rng(22)
    u = np.log(p.r) + 0.5 * rng.standard_normal(n)
    v = np.log(p.c) + 0.5 * rng.standard_normal(m)
    x = rng.standard_normal(n); y = rng.standard_normal(m)
    f, g = u * gamma, v * gamma
    u, v = O.to_log_units(f, g, gamma)
    say(f"high-d wide tiles n={n} m={m} d={d} {prec}")
    out = eot.eot_marginals(pc, gamma, dvec(f), dvec(g), precision=prec)
    Hx, Hy = eot.eot_hvp(pc, gamma, dvec(f), dvec(g), rho, dvec(x), dvec(y), precision=prec)
    torch.cuda.synchronize()
    rows = np.sort(rng.choice(n, 40, replace=False))
    cols = np.concatenate([np.sort(rng.choice(m, 36, replace=False)), [0, 2047, 2048, m - 1]])
    C_rows = O.sqeuclid_points_cost(p.X[rows], p.Y, p.scale)          # 40 x m
    C_cols = O.sqeuclid_points_cost(p.X, p.Y[cols], p.scale)          # n x 40
    tol = 1e-12 if prec == "fp64" else mixed_tol(beta)
    np.testing.assert_allclose(host(out["log_rP"])[rows], O.log_row_marginal(C_rows, beta, u[rows], v),
                               atol=tol, rtol=0)
    np.testing.assert_allclose(host(out["log_cP"])[cols], O.log_col_marginal(C_cols, beta, u, v[cols]),
                               atol=tol, rtol=0)
    hx_ref, _ = O.hvp(C_rows, beta, u[rows], v, rho, x[rows], y)
    ax, _ = O.hvp(C_rows, beta, u[rows], v, rho, np.abs(x[rows]), np.abs(y))
    _, hy_ref = O.hvp(C_cols, beta, u, v[cols], rho, x, y[cols])
    _, ay = O.hvp(C_cols, beta, u, v[cols], rho, np.abs(x), np.abs(y[cols]))
    assert np.all(np.abs(host(Hx)[rows] - hx_ref) <= tol * ax + 1e-300)
    assert np.all(np.abs(host(Hy)[cols] - hy_ref) <= tol * ay + 1e-300)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_highd_atomic_outputs_sampled(prec):
    """n = m = 65536, d = 64 (the benchmark's embedding size): the per-tile partials
    would exceed the library's limit, so the passes accumulate their outputs
    atomically. Marginals (with the row-maximum shift), the HVP and the mass
    identity, checked on sampled rows and columns against the oracle."""
    n = m = 1 << 16
    d, gamma, rho = 64, 0.05, 0.6
    beta = 1.0 / gamma
    p = W.embedding_problem(n, m, d, 31)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    rng = np.random.default_rng(32)
    u = np.log(p.r) + 0.5 * rng.standard_normal(n)
    v = np.log(p.c) + 0.5 * rng.standard_normal(m)
    x = rng.standard_normal(n); y = rng.standard_normal(m)
    f, g = u * gamma, v * gamma
    u, v = O.to_log_units(f, g, gamma)
    say(f"high-d atomic outputs n=m={n} d={d} {prec}")
    out = eot.eot_marginals(pc, gamma, dvec(f), dvec(g), precision=prec, want=("log_rP", "log_cP"))
    Hx, Hy = eot.eot_hvp(pc, gamma, dvec(f), dvec(g), rho, dvec(x), dvec(y), precision=prec)
    torch.cuda.synchronize()
    rows = np.concatenate([np.sort(rng.choice(n, 36, replace=False)), [0, n - 1]])
    cols = np.concatenate([np.sort(rng.choice(m, 36, replace=False)), [0, m - 1]])
    C_rows = O.sqeuclid_points_cost(p.X[rows], p.Y, p.scale)
    C_cols = O.sqeuclid_points_cost(p.X, p.Y[cols], p.scale)
    tol = 1e-12 if prec == "fp64" else mixed_tol(beta)
    lr, lc = host(out["log_rP"]), host(out["log_cP"])
    np.testing.assert_allclose(lr[rows], O.log_row_marginal(C_rows, beta, u[rows], v), atol=tol, rtol=0)
    np.testing.assert_allclose(lc[cols], O.log_col_marginal(C_cols, beta, u, v[cols]), atol=tol, rtol=0)
    m1 = np.exp(lr).sum(); m2 = np.exp(lc).sum()
    assert abs(m1 - m2) <= 10 * tol * m1
    hx_ref, _ = O.hvp(C_rows, beta, u[rows], v, rho, x[rows], y)
    ax, _ = O.hvp(C_rows, beta, u[rows], v, rho, np.abs(x[rows]), np.abs(y))
    _, hy_ref = O.hvp(C_cols, beta, u, v[cols], rho, x, y[cols])
    _, ay = O.hvp(C_cols, beta, u, v[cols], rho, np.abs(x), np.abs(y[cols]))
    assert np.all(np.abs(host(Hx)[rows] - hx_ref) <= tol * ax + 1e-300)
    assert np.all(np.abs(host(Hy)[cols] - hy_ref) <= tol * ay + 1e-300)


def test_highd_mixed_error_at_the_final_temperature():
    """The embedding workload's own temperatures (1/8 -> 1e-2, beta / scale = 25 at the
    end) at n = m = 2048, d = 64: a mixed solve, then the mixed log marginals at its
    output potentials against the oracle's. States the error the matrix-core form makes
    where the solve ends (the bound of the module docstring, 1.2e-3 at beta = 100), and
    that the solve still reaches its tolerance: the mixed projections that stall at that
    floor hand over to FP64 (R18), the last one always finishes in FP64."""
    p, pc, C = cloud(2048, 2048, 64, 77)
    gamma = p.gamma_final
    beta = 1.0 / gamma
    f, g, st = eot.eot_solve(pc, dvec(p.r), dvec(p.c), gamma_init=p.gamma_init,
                             gamma_final=gamma, tol=p.tol, precision="mixed")
    assert st["status"] == 0 and st["err_r"] + st["err_c"] <= p.tol
    u, v = O.to_log_units(host(f), host(g), gamma)
    lr_ref = O.log_row_marginal(C, beta, u, v)
    lc_ref = O.log_col_marginal(C, beta, u, v)
    res = {}
    for prec in ("mixed", "fp64"):
        out = eot.eot_marginals(pc, gamma, f, g, precision=prec, want=("log_rP", "log_cP"))
        torch.cuda.synchronize()
        res[prec] = max(np.abs(host(out["log_rP"]) - lr_ref).max(),
                        np.abs(host(out["log_cP"]) - lc_ref).max())
    say(f"embeddings 2048 x 2048, d = 64, solve at gamma {gamma:g} (beta {beta:g}): log-marginal "
        f"error against the oracle mixed {res['mixed']:.2e} (bound {mixed_tol(beta):.1e}), "
        f"fp64 {res['fp64']:.1e}; solve error {st['err_r'] + st['err_c']:.1e}, mixed stalls "
        f"{st['mixed_stalls']}, range retries {st['range_retries']}")
    assert res["mixed"] <= mixed_tol(beta)
    assert res["fp64"] <= 1e-12 + 2.0 ** -52 * beta * C.max()
