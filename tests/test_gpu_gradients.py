"""GPU parity of eot_gradient (W and S derivatives) and of the autograd
wrappers against the oracle's derivative formulas (oracle/gradients.py,
pinned by finite differences), evaluated at the GPU potentials.

Tolerances: the cotangent G and the marginal gradients are compared with
1e-8 of their largest entry. The S part goes through the CG solve of
H [lam; mu] = [a; b] to a relative L1 residual of 1e-11; lam then carries
that residual times the conditioning of the Schur complement on the
complement of its null vector, < 1e3 for these temperatures, hence 1e-8.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import gradients as OG
from paper_2504_02067_amd import autograd as AG
from paper_2504_02067_amd import eot
from paper_2504_02067_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(msg):
    print(f"[gpu-grad] {msg}", flush=True)


def dvec(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def close(a, b, rel=1e-8):
    scale = max(np.abs(b).max(), 1e-300)
    assert np.abs(a - b).max() <= rel * scale, (np.abs(a - b).max() / scale)


def dense_case(n, m, seed, gamma):
    rng = np.random.default_rng(seed)
    C = rng.uniform(0, 1, size=(n, m)).astype(np.float32)
    r = rng.dirichlet(np.ones(n)) + 1e-3; r /= r.sum()
    c = rng.dirichlet(np.ones(m)) + 1e-3; c /= c.sum()
    Cd = torch.from_numpy(C).to(DEV)
    f, g, st = eot.eot_solve(Cd, dvec(r), dvec(c), gamma_init=1.0 / 8.0, gamma_final=gamma,
                             tol=1e-9, precision="fp64")
    return C, Cd, r, c, f, g, st


@pytest.mark.parametrize("w_W,w_S", [(1.0, 0.0), (0.0, 1.0), (0.7, -1.3)])
@pytest.mark.parametrize("n,m", [(150, 230), (300, 2100)])
def test_dense_gradient_parity(n, m, w_W, w_S):
    gamma = 0.05
    C, Cd, r, c, f, g, st = dense_case(n, m, n + m, gamma)
    say(f"dense gradient n={n} m={m} wW={w_W} wS={w_S}")
    out = eot.eot_gradient(Cd, gamma, f, g, w_W=w_W, w_S=w_S)
    u, v = O.to_log_units(host(f), host(g), gamma)
    beta = 1.0 / gamma
    G, gr, gc, S, lam, mu = OG.vjp(C, beta, u, v, w_W, w_S)
    say(f"  cg_iters={out['cg_iters']} residual={out['cg_residual']:.2e}")
    assert abs(out["S"] - S) <= 1e-12 * S
    close(host(out["C"]), G)
    close(host(out["r"]), gr)
    close(host(out["c"]), gc)


@pytest.mark.parametrize("d", [2, 3])
def test_points_gradient_parity(d):
    gamma = 0.02
    p = W.point_cloud_problem(n=400, m=530, d=d, seed=70 + d)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    f, g, st = eot.eot_solve(pc, dvec(p.r), dvec(p.c), gamma_init=1.0 / 8.0, gamma_final=gamma,
                             tol=1e-9, precision="fp64")
    say(f"points gradient d={d}")
    out = eot.eot_gradient(pc, gamma, f, g, w_W=0.4, w_S=1.1)
    C = O.sqeuclid_points_cost(p.X, p.Y, p.scale)
    u, v = O.to_log_units(host(f), host(g), gamma)
    G, gr, gc, S, _, _ = OG.vjp(C, 1.0 / gamma, u, v, 0.4, 1.1)
    gX, gY = OG.points_grad(p.X, p.Y, p.scale, G)
    assert abs(out["S"] - S) <= 1e-12 * S
    close(host(out["X"]), gX)
    close(host(out["Y"]), gY)
    close(host(out["r"]), gr)
    close(host(out["c"]), gc)


def test_points_and_dense_paths_agree_on_a_grid():
    """Grid positions as points (d = 2, 4096 points) against the dense grid
    cost: the dense cotangent pushed through the chain rule must give the
    point gradient."""
    side = 64
    p = W.batch_problem(0, sides=np.array([side]))
    gamma = 1e-2
    Cd = torch.from_numpy(W.grid_cost(side, "sqeuclid", np.float64)).to(DEV)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    f, g, st = eot.eot_solve(Cd, dvec(p.r), dvec(p.c), gamma_init=1.0 / 8.0, gamma_final=gamma,
                             tol=1e-9, precision="fp64")
    say("grid 64x64: dense vs points gradient")
    a = eot.eot_gradient(Cd, gamma, f, g, w_W=1.0, w_S=0.5, want=("C", "r"))
    b = eot.eot_gradient(pc, gamma, f, g, w_W=1.0, w_S=0.5, want=("X", "Y", "r"))
    Gd = host(a["C"])
    gX, gY = OG.points_grad(p.X, p.Y, p.scale, Gd)
    close(host(b["X"]), gX, 1e-9)
    close(host(b["Y"]), gY, 1e-9)
    close(host(b["r"]), host(a["r"]), 1e-9)


def test_autograd_dense_matches_finite_differences():
    gamma = 0.1
    n, m = 40, 50
    rng = np.random.default_rng(8)
    C = torch.from_numpy(rng.uniform(0, 1, size=(n, m))).to(DEV).requires_grad_(True)
    r = dvec(np.full(n, 1.0 / n)).requires_grad_(True)
    c = dvec(rng.dirichlet(np.ones(m)) * 0.5 + 0.5 / m)
    kw = dict(gamma_init=gamma, tol=1e-13, grad_tol=1e-12)
    Wv, Sv = AG.entropic_ot(C, r, c, gamma, **kw)
    loss = 0.3 * Wv + 2.0 * Sv
    loss.backward()
    gC = host(C.grad)
    gr = host(r.grad)
    say("autograd dense vs finite differences")
    # S moves to first order with the potentials' residual error (tol 1e-13),
    # so the step is 1e-4: noise < 1e-9, truncation ~ h^2 beta^3 P ~ 1e-9
    h = 1e-4
    for (i, j) in [(0, 0), (17, 33), (39, 49)]:
        E = torch.zeros_like(C); E[i, j] = h
        Wp, Sp = AG.entropic_ot((C + E).detach(), r.detach(), c, gamma, **kw)
        Wm, Sm = AG.entropic_ot((C - E).detach(), r.detach(), c, gamma, **kw)
        fd = (0.3 * (Wp - Wm) + 2.0 * (Sp - Sm)).item() / (2 * h)
        assert fd == pytest.approx(gC[i, j], rel=1e-5, abs=1e-9)
    dr = rng.standard_normal(n); dr -= dr.mean()
    drt = dvec(dr)
    Wp, Sp = AG.entropic_ot(C.detach(), (r + h * drt).detach(), c, gamma, **kw)
    Wm, Sm = AG.entropic_ot(C.detach(), (r - h * drt).detach(), c, gamma, **kw)
    fd = (0.3 * (Wp - Wm) + 2.0 * (Sp - Sm)).item() / (2 * h)
    assert fd == pytest.approx(gr @ dr, rel=1e-5, abs=1e-9)


def test_autograd_points_backward_runs_the_library():
    gamma = 0.05
    p = W.point_cloud_problem(n=300, m=300, d=3, seed=31)
    X = torch.from_numpy(p.X).to(DEV).requires_grad_(True)
    Y = torch.from_numpy(p.Y).to(DEV).requires_grad_(True)
    Wv, Sv = AG.entropic_ot_points(X, Y, dvec(p.r), dvec(p.c), gamma, p.scale,
                                   gamma_init=1.0 / 8.0, tol=1e-9)
    Sv.backward()
    assert X.grad.dtype == torch.float32 and X.grad.shape == X.shape
    C = O.sqeuclid_points_cost(p.X, p.Y, p.scale)
    f, g, st = eot.eot_solve(eot.PointCloud(X.detach(), Y.detach(), p.scale), dvec(p.r),
                             dvec(p.c), gamma_init=1.0 / 8.0, gamma_final=gamma, tol=1e-9)
    u, v = O.to_log_units(host(f), host(g), gamma)
    G, *_ = OG.vjp(C, 1.0 / gamma, u, v, 0.0, 1.0)
    gX, gY = OG.points_grad(p.X, p.Y, p.scale, G)
    say("autograd points")
    close(host(X.grad).astype(np.float64), gX, 1e-6)
    close(host(Y.grad).astype(np.float64), gY, 1e-6)


# ---------------------------------------------------------------- rounding

@pytest.mark.parametrize("n,m,prec", [(150, 230, "fp64"), (300, 2100, "mixed"), (1, 7, "fp64")])
def test_round_parity(n, m, prec):
    gamma = 0.05
    rng = np.random.default_rng(n * m)
    C = rng.uniform(0, 1, size=(n, m)).astype(np.float32)
    r = rng.dirichlet(np.ones(n)) + 1e-3; r /= r.sum()
    c = rng.dirichlet(np.ones(m)) + 1e-3; c /= c.sum()
    Cd = torch.from_numpy(C).to(DEV)
    f, g, st = eot.eot_solve(Cd, dvec(r), dvec(c), gamma_init=1.0 / 8.0, gamma_final=gamma,
                             tol=1e-4, precision=prec)
    say(f"round n={n} m={m}")
    out = eot.eot_round(Cd, gamma, f, g, dvec(r), dvec(c), plan=True)
    u, v = O.to_log_units(host(f), host(g), gamma)
    Pr = O.round_plan(C, 1.0 / gamma, u, v, r, c)
    X = host(out["plan"])
    # the deficits er = r - r(D(x) P D(y)) and ec cancel (they are ~tol of r and
    # c), so their rounding, O(1e-16) of r_i and c_j, reaches the rank-one
    # correction er_i ec_j / |er|_1 as ~1e-16 r_i c_j / |er|_1
    nr = max(out["mass_fix"], 1e-300)
    bound = 1e-12 * np.abs(Pr) + 1e-13 * np.outer(r, c) / nr
    assert np.all(np.abs(X - Pr) <= bound)
    np.testing.assert_allclose(X.sum(1), r, rtol=1e-12)
    np.testing.assert_allclose(X.sum(0), c, rtol=1e-12)
    Cd64 = C.astype(np.float64)
    assert out["cost_round"] == pytest.approx((Pr * Cd64).sum(), rel=1e-12)
    P = OG.plan(C, 1.0 / gamma, u, v)
    assert out["cost_plan"] == pytest.approx((P * Cd64).sum(), rel=1e-12)
    assert out["err_r"] == pytest.approx(np.abs(P.sum(1) - r).sum(), rel=1e-9, abs=1e-15)
    # the implicit form gives the same matrix
    Xi = (host(out["x"])[:, None] * P * host(out["y"])[None, :]
          + np.outer(host(out["er"]), host(out["ec"])) / max(out["mass_fix"], 1e-300))
    assert np.all(np.abs(Xi - Pr) <= bound)


def test_round_points_cost_matches_dense():
    gamma = 0.02
    p = W.point_cloud_problem(n=500, m=300, d=3, seed=90)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    f, g, st = eot.eot_solve(pc, dvec(p.r), dvec(p.c), gamma_init=1.0 / 8.0, gamma_final=gamma,
                             tol=1e-3)
    say("round points")
    out = eot.eot_round(pc, gamma, f, g, dvec(p.r), dvec(p.c))
    C = O.sqeuclid_points_cost(p.X, p.Y, p.scale)
    u, v = O.to_log_units(host(f), host(g), gamma)
    Pr = O.round_plan(C, 1.0 / gamma, u, v, p.r, p.c)
    assert out["cost_round"] == pytest.approx((Pr * C).sum(), rel=1e-11)


def test_autograd_points_matches_finite_differences():
    """d(0.3 W + 2 S)/dX and /dY of GPU solves against central differences of GPU
    solves; coordinates on a 2^-10 grid and a step of 2^-8, so X +- h is exact in
    FP32."""
    gamma = 0.1
    rng = np.random.default_rng(21)
    n, m, d = 30, 40, 2
    Xh = np.round(rng.uniform(0, 1, (n, d)) * 1024) / 1024
    Yh = np.round(rng.uniform(0, 1, (m, d)) * 1024) / 1024
    scale = 2.0
    r = dvec(np.full(n, 1.0 / n)); c = dvec(np.full(m, 1.0 / m))
    kw = dict(gamma_init=gamma, tol=1e-13, grad_tol=1e-12)

    def loss(X, Y):
        Wv, Sv = AG.entropic_ot_points(X, Y, r, c, gamma, scale, **kw)
        return 0.3 * Wv + 2.0 * Sv

    X = torch.from_numpy(Xh.astype(np.float32)).to(DEV).requires_grad_(True)
    Y = torch.from_numpy(Yh.astype(np.float32)).to(DEV).requires_grad_(True)
    loss(X, Y).backward()
    gX, gY = host(X.grad).astype(np.float64), host(Y.grad).astype(np.float64)
    say("autograd points vs finite differences")
    h = 2.0 ** -8
    for (T, G, idx) in ((X, gX, [(0, 0), (17, 1), (29, 0)]), (Y, gY, [(3, 1), (39, 0)])):
        for (i, k) in idx:
            E = torch.zeros_like(T); E[i, k] = h
            if T is X:
                fd = (loss((X + E).detach(), Y.detach()) - loss((X - E).detach(), Y.detach())).item()
            else:
                fd = (loss(X.detach(), (Y + E).detach()) - loss(X.detach(), (Y - E).detach())).item()
            fd /= 2 * h
            assert fd == pytest.approx(G[i, k], rel=2e-3, abs=1e-5)


def test_gradient_mixed_cg_matches_fp64():
    gamma = 0.05
    C, Cd, r, c, f, g, st = dense_case(300, 200, 5, gamma)
    say("gradient with mixed-precision CG")
    a = eot.eot_gradient(Cd, gamma, f, g, w_W=0.5, w_S=1.0)
    b = eot.eot_gradient(Cd, gamma, f, g, w_W=0.5, w_S=1.0, precision="mixed", tol=1e-6)
    # the CG solve stops at a 1e-6 relative residual in FP32-plan passes: lam, mu to ~1e-5
    close(host(b["C"]), host(a["C"]), 1e-4)
    close(host(b["r"]), host(a["r"]), 1e-4)
    assert b["S"] == pytest.approx(a["S"], rel=1e-12)


def test_round_fp64_cost():
    gamma = 0.1
    rng = np.random.default_rng(3)
    C = rng.uniform(0, 1, (90, 70))
    r = rng.dirichlet(np.ones(90)); c = rng.dirichlet(np.ones(70))
    Cd = torch.from_numpy(C).to(DEV)
    f, g, _ = eot.eot_solve(Cd, dvec(r), dvec(c), gamma_init=gamma, gamma_final=gamma, tol=1e-3)
    out = eot.eot_round(Cd, gamma, f, g, dvec(r), dvec(c), plan=True)
    u, v = O.to_log_units(host(f), host(g), gamma)
    Pr = O.round_plan(C, 1 / gamma, u, v, r, c)
    nr = max(out["mass_fix"], 1e-300)
    assert np.all(np.abs(host(out["plan"]) - Pr) <= 1e-12 * np.abs(Pr) + 1e-13 * np.outer(r, c) / nr)
    assert out["cost_round"] == pytest.approx((Pr * C).sum(), rel=1e-12)


def test_nonfinite_cost_is_reported():
    """A NaN in the cost ends the solve with EOT_ERR_NONFINITE instead of a
    silent result (the passes' range guard sees the non-finite sums)."""
    rng = np.random.default_rng(4)
    C = rng.uniform(0, 1, (64, 64)).astype(np.float32)
    C[10, 20] = np.nan
    r = np.full(64, 1 / 64); c = np.full(64, 1 / 64)
    say("NaN cost")
    with pytest.raises(eot.EotError) as e:
        eot.eot_solve(torch.from_numpy(C).to(DEV), dvec(r), dvec(c), gamma_init=0.1,
                      gamma_final=0.01, tol=1e-6, max_mdot=20)
    assert e.value.status == eot.EOT_ERR_NONFINITE
