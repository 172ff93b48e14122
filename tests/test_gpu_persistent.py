"""The persistent batched solver (eot_solve_batched with batch_persistent = 1):
every problem of the batch solved by one cooperative launch per cost kind,
teams of workgroups running MDOT / TruncatedNewtonProject / NewtonSolve / CG /
the line search on the device. Checked against the FP64 oracle problem by
problem: FP64 mode takes the oracle's MDOT and Newton steps and reaches its
transport cost within 1e-10; mixed precision reaches it within 1e-5 at the
same final marginal error bound. Team sizes 1 (tiny problems), 2-4 and 8
(the 1024-bin problems) all occur below, so both the workgroup-only and the
cross-workgroup barrier paths run. Also: cost kinds mixed in one call, a
failing problem that does not stop the others, and run-to-run reproducibility
(fixed summation orders)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2504_02067_amd import eot
from paper_2504_02067_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
KW = dict(gamma_init=1.0 / 32.0, gamma_final=1e-3, tol=1e-6)


def say(msg):
    print(f"[gpu-persistent] {msg}", flush=True)


def dvec(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def grid_batch(count, lo, hi, seed):
    sides = W.batch_sides(seed, count, lo, hi)
    probs, items = [], []
    for k in range(count):
        p = W.batch_problem(k, seed, sides)
        pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
        probs.append(p)
        items.append((pc, dvec(p.r), dvec(p.c)))
    return probs, items


def oracle_of(p, **kw):
    # the GPU sees the points (the cost recomputed from them), so the oracle does too
    C = O.sqeuclid_points_cost(p.X, p.Y, p.scale)
    return O.solve(C, p.r, p.c, **kw)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_persistent_grid_batch_against_oracle(prec):
    """8 grid problems, sides 16..32 (256..1024 bins; the 1024-bin ones run
    on teams of 8 workgroups)."""
    probs, items = grid_batch(8, 16, 32, 4500)
    say(f"persistent batch of 8 ({prec}), n = {[p.n for p in probs]}")
    outs, stats, status = eot.eot_solve_batched(items, precision=prec, **KW)
    assert status == [0] * len(items)
    for k, p in enumerate(probs):
        u, v, ost = oracle_of(p, **KW)
        st = stats[k]
        rel = abs(st["cost"] - ost["cost"]) / ost["cost"]
        say(f"  n={p.n}: cost rel {rel:.2e}, newton {st['newton_steps']}/{ost['newton_steps']}, "
            f"mdot {st['mdot_steps']}/{ost['mdot_steps']}, cg {st['cg_iters']}/{ost['cg_iters']}, "
            f"err {st['err_r'] + st['err_c']:.2e}")
        assert st["err_r"] + st["err_c"] <= KW["tol"]
        if prec == "fp64":
            assert rel <= 1e-10
            assert st["mdot_steps"] == ost["mdot_steps"]
            assert st["newton_steps"] == ost["newton_steps"]
        else:
            assert rel <= 1e-5
        # the potentials returned re-evaluate to the reported error
        f, g = outs[k]
        beta = 1.0 / KW["gamma_final"]
        C = O.sqeuclid_points_cost(p.X, p.Y, p.scale)
        gu, gv = f.cpu().numpy() * beta, g.cpu().numpy() * beta
        er = np.abs(np.exp(O.log_row_marginal(C, beta, gu, gv)) - p.r).sum()
        ec = np.abs(np.exp(O.log_col_marginal(C, beta, gu, gv)) - p.c).sum()
        assert er + ec <= KW["tol"]


def test_persistent_cost_kinds_in_one_call():
    """Dense FP32 (28 x 28 grid, L1 and squared L2), dense FP64 (64 points),
    3-D points and 2-D points in one call, FP64, each against the oracle."""
    items, refs = [], []
    for kind in ("l1", "sqeuclid"):
        p = W.mnist_like_problem(2000, kind)
        items.append((torch.from_numpy(p.C).to(DEV), dvec(p.r), dvec(p.c)))
        refs.append((p, p.C))
    for seed in (1000, 1001):
        p = W.small_points_problem(seed)
        items.append((dvec(p.C), dvec(p.r), dvec(p.c)))
        refs.append((p, p.C))
    p3 = W.point_cloud_problem(n=300, m=200, seed=77)
    items.append((eot.PointCloud(torch.from_numpy(p3.X).to(DEV), torch.from_numpy(p3.Y).to(DEV),
                                 p3.scale), dvec(p3.r), dvec(p3.c)))
    refs.append((p3, O.sqeuclid_points_cost(p3.X, p3.Y, p3.scale)))
    kw = dict(gamma_init=1.0 / 32.0, gamma_final=1e-3, tol=1e-6)
    say("persistent batch of mixed kinds (fp64)")
    outs, stats, status = eot.eot_solve_batched(items, precision="fp64", **kw)
    assert status == [0] * len(items)
    for k, (p, C) in enumerate(refs):
        kwp = dict(kw)
        if p.name.startswith("grid28"):
            kwp.update(gamma_init=p.gamma_init, gamma_final=p.gamma_final, tol=p.tol)
        if k < 2:   # the grid problems use their own schedule: solve them again with it
            continue
        u, v, ost = O.solve(C, p.r, p.c, **kwp)
        rel = abs(stats[k]["cost"] - ost["cost"]) / ost["cost"]
        say(f"  {p.name}: cost rel {rel:.2e}, newton {stats[k]['newton_steps']}/{ost['newton_steps']}")
        assert rel <= 1e-10 and stats[k]["newton_steps"] == ost["newton_steps"]
    # the 28 x 28 grids on their own schedule (temperature 1/32 -> 1e-4)
    for k in (0, 1):
        p, C = refs[k]
        kwp = dict(gamma_init=p.gamma_init, gamma_final=p.gamma_final, tol=p.tol)
        o2, s2, st2 = eot.eot_solve_batched([items[k]], precision="fp64", **kwp)
        u, v, ost = O.solve(C, p.r, p.c, **kwp)
        rel = abs(s2[0]["cost"] - ost["cost"]) / ost["cost"]
        say(f"  {p.name}: cost rel {rel:.2e}, newton {s2[0]['newton_steps']}/{ost['newton_steps']}, "
            f"misses {s2[0]['forcing_misses']}/{ost['forcing_misses']}")
        assert st2 == [0] and s2[0]["err_r"] + s2[0]["err_c"] <= p.tol
        assert s2[0]["mdot_steps"] == ost["mdot_steps"]
        if ost["forcing_misses"] == 0:
            assert rel <= 1e-10 and s2[0]["newton_steps"] == ost["newton_steps"]
        else:
            # NewtonSolve at the discount cap (nearly decomposable plan): CG at a
            # condition number up to ~2e9 depends on the summation order, so the
            # trajectories part (as for the host path's trace, test_gpu_trace.py);
            # both end within the tolerance, a few Newton steps apart
            assert abs(s2[0]["newton_steps"] - ost["newton_steps"]) <= 0.1 * ost["newton_steps"]
            assert rel <= 1e-8


def test_persistent_failure_isolation_and_reproducibility():
    probs, items = grid_batch(5, 16, 24, 4600)
    bad_r = dvec(np.full(probs[1].n, 2.0 / probs[1].n))          # sums to 2
    items.insert(2, (items[1][0], bad_r, items[1][2]))
    say("persistent batch with one invalid problem, twice")
    o1, s1, st1 = eot.eot_solve_batched(items, precision="mixed", check=False, **KW)
    o2, s2, st2 = eot.eot_solve_batched(items, precision="mixed", check=False, **KW)
    assert st1[2] == eot.EOT_ERR_BAD_MARGINALS and st2 == st1
    assert [s for k, s in enumerate(st1) if k != 2] == [0] * (len(items) - 1)
    for k in range(len(items)):
        if k == 2:
            continue
        assert torch.equal(o1[k][0], o2[k][0]) and torch.equal(o1[k][1], o2[k][1]), k
        assert s1[k]["cg_iters"] == s2[k]["cg_iters"]


def test_persistent_and_host_paths_take_the_same_steps():
    """FP64: the persistent solver and the host-driven one make the same
    decisions (both are the oracle's)."""
    probs, items = grid_batch(6, 16, 28, 4700)
    say("persistent vs host workers (fp64)")
    _, sp, stp = eot.eot_solve_batched(items, precision="fp64", **KW)
    _, sh, sth = eot.eot_solve_batched(items, precision="fp64", batch_persistent=0, **KW)
    assert stp == sth == [0] * len(items)
    for k in range(len(items)):
        assert sp[k]["mdot_steps"] == sh[k]["mdot_steps"]
        assert sp[k]["newton_steps"] == sh[k]["newton_steps"]
        assert abs(sp[k]["cost"] - sh[k]["cost"]) <= 1e-10 * sh[k]["cost"]
