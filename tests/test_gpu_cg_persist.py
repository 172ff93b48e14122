"""The single-launch CG of small problems (launch_cg_persist: one cooperative
kernel per CG solve of NewtonSolve, Alg. 2, parity-tagged exchange between
its workgroups)
against the launches-per-iteration path it replaces (eot_set_cg_persist(0)),
which the other GPU tests pin to the oracle: the same NewtonSolve directions
(the summation orders differ, so to rounding), the same CG iteration counts,
and full solves that take the same steps and reach the same cost; on dense FP32
/ FP64 costs and on 2-D / 3-D points, square and ragged, at the size limit and
just past it (where the launches per iteration take over), and for several
grid sizes (which change only the block sums' grouping)."""
import numpy as np
import pytest
import torch

from paper_2504_02067_amd import eot
from paper_2504_02067_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(msg):
    print(f"[gpu-cg-persist] {msg}", flush=True)


def dvec(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(autouse=True)
def _restore():
    yield
    eot.eot_set_cg_persist(1, 0)


def newton_both(C, gamma, f, g, r, c, prec, grid=0, eta=0.05, rho0=0.0):
    out = {}
    for mode in (0, 1):
        eot.eot_set_cg_persist(mode, grid if mode else 0)
        o = eot.eot_newton_cg(C, gamma, f, g, r, c, eta, rho0, precision=prec)
        torch.cuda.synchronize()
        out[mode] = o
    return out[0], out[1]


def fixed_point(p, C, prec):
    """Potentials where c(P) = c at the problem's first temperature (a short
    solve there), so NewtonSolve starts from the state Alg. 4 gives it."""
    f, g, st = eot.eot_solve(C, dvec(p.r), dvec(p.c), gamma_init=p.gamma_init,
                             gamma_final=p.gamma_init * 0.5, tol=1e-3, precision=prec,
                             allow_not_converged=True)
    return f, g


def check_dirs(a, b, prec, where, ref=None):
    """a: launches per iteration, b: single launch. FP64: equal to rounding.
    Mixed: the two paths round their plan entries differently (hi / lo FP32
    assembly against an FP64 exponent rounded once), which the CG amplifies by
    the discounted system's condition number; so each is compared with the
    FP64 direction `ref`, and the single launch must be as close as the
    launches per iteration (within 3x, or 1e-6 relative)."""
    for name in ("dir_f", "dir_g"):
        x, y = host(getattr(a, name)), host(getattr(b, name))
        scale = np.abs(x).max()
        err = np.abs(x - y).max() / scale
        say(f"{where} {name}: rel diff {err:.2e}, cg {a.cg_iters}/{b.cg_iters}, "
            f"levels {a.levels}/{b.levels}")
        if prec == "fp64":
            assert err <= 1e-9, (where, name, err)
        else:
            z = host(getattr(ref, name))
            ea = np.abs(x - z).max() / np.abs(z).max()
            eb = np.abs(y - z).max() / np.abs(z).max()
            say(f"{where} {name}: vs FP64 {ea:.2e} (launches) {eb:.2e} (single launch)")
            assert eb <= max(3.0 * ea, 1e-6), (where, name, ea, eb)
    if prec == "fp64":
        assert abs(a.cg_iters - b.cg_iters) <= max(1, a.cg_iters // 50), where
        assert a.levels == b.levels and a.forcing_miss == b.forcing_miss, where
    else:
        assert abs(a.cg_iters - b.cg_iters) <= max(2, a.cg_iters // 10), where
        assert abs(a.levels - b.levels) <= 1, where


@pytest.mark.parametrize("kind", ["sqeuclid", "l1"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_newton_direction_dense_grid28(kind, prec):
    p = W.mnist_like_problem(2000, kind)
    C = torch.from_numpy(p.C).to(DEV)
    f, g = fixed_point(p, C, prec)
    gamma = p.gamma_init * 0.5
    a, b = newton_both(C, gamma, f, g, dvec(p.r), dvec(p.c), prec)
    ref = newton_both(C, gamma, f, g, dvec(p.r), dvec(p.c), "fp64")[0] if prec == "mixed" else None
    check_dirs(a, b, prec, f"grid28 {kind} {prec}", ref)


@pytest.mark.parametrize("d", [2, 3])
# (130, 1000): 125 workgroups over 130 rows, one or two each; (100, 900): no
# grid has both at most 8 columns and at least one row per workgroup, so both
# modes take the launches per iteration
@pytest.mark.parametrize("nm", [(300, 517), (1024, 1024), (1025, 700), (130, 1000), (100, 900)])
def test_newton_direction_points(d, nm):
    n, m = nm
    rng = np.random.default_rng(d * 1000 + n)
    X = rng.uniform(0, 1, (n, d)).astype(np.float32)
    Y = rng.uniform(0, 1, (m, d)).astype(np.float32)
    pc = eot.PointCloud(torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV), float(d))
    r = rng.dirichlet(np.ones(n)) * 0.5 + 0.5 / n
    c = rng.dirichlet(np.ones(m)) * 0.5 + 0.5 / m
    f, g, _ = eot.eot_solve(pc, dvec(r), dvec(c), gamma_init=0.1, gamma_final=0.02, tol=1e-4,
                            precision="fp64", allow_not_converged=True)
    ref = None
    for prec in ("fp64", "mixed"):
        a, b = newton_both(pc, 0.02, f, g, dvec(r), dvec(c), prec, rho0=0.75)
        check_dirs(a, b, prec, f"points d={d} {n}x{m} {prec}", ref)
        ref = a


def test_newton_direction_dense_fp64_cost_and_grid_sizes():
    rng = np.random.default_rng(11)
    n, m = 640, 384
    C = rng.uniform(0, 1, (n, m))
    r = rng.dirichlet(np.ones(n)) * 0.5 + 0.5 / n
    c = rng.dirichlet(np.ones(m)) * 0.5 + 0.5 / m
    Cd = dvec(C)
    f, g, _ = eot.eot_solve(Cd, dvec(r), dvec(c), gamma_init=0.1, gamma_final=0.01, tol=1e-4,
                            precision="fp64", allow_not_converged=True)
    ref = None
    for grid in (3, 80, 101, 128):                # 3 is raised to max(n, m) / 8 = 80
        a, b = newton_both(Cd, 0.01, f, g, dvec(r), dvec(c), "fp64", grid=grid, rho0=0.75)
        check_dirs(a, b, "fp64", f"dense FP64 640x384 grid {grid}")
        if ref is not None:
            assert np.abs(host(b.dir_f) - host(ref.dir_f)).max() <= 1e-9 * np.abs(host(ref.dir_f)).max()
        ref = b


@pytest.mark.parametrize("kind", ["sqeuclid", "l1"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_grid28_same_steps(kind, prec):
    p = W.mnist_like_problem(2001, kind)
    C = torch.from_numpy(p.C).to(DEV)
    res = {}
    for mode in (0, 1):
        eot.eot_set_cg_persist(mode, 0)
        _, _, st = eot.eot_solve(C, dvec(p.r), dvec(p.c), gamma_init=p.gamma_init,
                                 gamma_final=p.gamma_final, tol=p.tol, precision=prec)
        res[mode] = st
    a, b = res[0], res[1]
    say(f"grid28 {kind} {prec}: newton {a['newton_steps']}/{b['newton_steps']} cg "
        f"{a['cg_iters']}/{b['cg_iters']} cost {a['cost']:.12f}/{b['cost']:.12f} "
        f"seconds {a['seconds']:.3f}/{b['seconds']:.3f}")
    assert a["status"] == 0 and b["status"] == 0
    assert b["err_r"] + b["err_c"] <= p.tol
    assert a["mdot_steps"] == b["mdot_steps"]
    # L1 at beta 1e4 takes the rounding-sensitive capped-discount path (R7)
    lim = 0.1 if kind == "l1" else 0.02
    assert abs(a["newton_steps"] - b["newton_steps"]) <= max(1, lim * a["newton_steps"])
    assert abs(a["cost"] - b["cost"]) <= (1e-8 if kind == "l1" else 1e-10) * abs(a["cost"])
