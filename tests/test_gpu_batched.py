"""GPU tests of eot_solve_batched on its host-worker path (batch_persistent =
0): the ragged grid batch (integer grid positions as 2-D points, cost
recomputed on the fly) solved concurrently must give bitwise the potentials of
solving each problem alone; mixed cost kinds share one batch; a failing
problem does not stop the others; and sampled problems match the oracle. The
persistent single-launch path is tested in test_gpu_persistent.py."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2504_02067_amd import eot
from paper_2504_02067_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _launches_per_iteration():
    """The batch workers (and the CG graph replay) launch each CG iteration;
    the single solves they are compared with bitwise do the same here."""
    eot.eot_set_cg_persist(0, 0)
    yield
    eot.eot_set_cg_persist(1, 0)


def say(msg):
    print(f"[gpu-batch] {msg}", flush=True)


def dvec(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def batch(count, lo=16, hi=40, seed=4000):
    sides = W.batch_sides(seed, count, lo, hi)
    probs, items = [], []
    for k in range(count):
        p = W.batch_problem(k, seed, sides)
        pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
        probs.append(p)
        items.append((pc, dvec(p.r), dvec(p.c)))
    return probs, items


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_equals_one_by_one(prec):
    probs, items = batch(24)
    opts = dict(gamma_init=1.0 / 32.0, gamma_final=1e-3, tol=1e-6, precision=prec,
                batch_persistent=0)
    say(f"batch of 24 ({prec}), 4 workers")
    outs, stats, status = eot.eot_solve_batched(items, workers=4, **opts)
    assert all(s == 0 for s in status)
    for k, (pc, r, c) in enumerate(items):
        f, g, st = eot.eot_solve(pc, r, c, **opts)
        assert torch.equal(outs[k][0], f) and torch.equal(outs[k][1], g), k
        assert stats[k]["newton_steps"] == st["newton_steps"]
        assert stats[k]["cg_iters"] == st["cg_iters"]
        assert stats[k]["err_r"] + stats[k]["err_c"] <= 1e-6


def test_batched_matches_oracle_on_samples():
    probs, items = batch(6, lo=16, hi=24, seed=4100)
    say("batch of 6 vs oracle")
    outs, stats, status = eot.eot_solve_batched(items, workers=3, gamma_init=1.0 / 32.0,
                                                gamma_final=1e-3, tol=1e-6, batch_persistent=0)
    for k in (0, 3, 5):
        p = probs[k]
        C = O.sqeuclid_points_cost(p.X, p.Y, p.scale)
        u, v, ost = O.solve(C, p.r, p.c, gamma_init=1.0 / 32.0, gamma_final=1e-3, tol=1e-6)
        assert abs(stats[k]["cost"] - ost["cost"]) <= 1e-10 * ost["cost"]
        assert stats[k]["newton_steps"] == ost["newton_steps"]


def test_batched_mixed_kinds_and_failure_isolation():
    rng = np.random.default_rng(9)
    items = []
    for n, m in ((300, 200), (64, 64), (1000, 700)):
        C = torch.from_numpy(rng.uniform(0, 1, (n, m)).astype(np.float32)).to(DEV)
        items.append((C, dvec(rng.dirichlet(np.ones(n))), dvec(rng.dirichlet(np.ones(m)))))
    probs, pitems = batch(3, seed=4200)
    items += pitems
    bad_r = dvec(np.full(64, 2.0 / 64))                    # sums to 2: rejected
    items.insert(2, (items[1][0], bad_r, items[1][2]))
    say("mixed kinds with one invalid problem")
    with pytest.raises(eot.EotError) as e:
        eot.eot_solve_batched(items, workers=4, gamma_init=0.1, gamma_final=1e-2, tol=1e-6,
                              batch_persistent=0)
    assert e.value.status == eot.EOT_ERR_BAD_MARGINALS
    outs, stats, status = eot.eot_solve_batched(items, workers=4, gamma_init=0.1,
                                                gamma_final=1e-2, tol=1e-6, check=False,
                                                batch_persistent=0)
    assert status[2] == eot.EOT_ERR_BAD_MARGINALS
    assert [s for k, s in enumerate(status) if k != 2] == [0] * (len(items) - 1)
    for k, (C, r, c) in enumerate(items):
        if k == 2:
            continue
        f, g, st = eot.eot_solve(C, r, c, gamma_init=0.1, gamma_final=1e-2, tol=1e-6)
        assert torch.equal(outs[k][0], f) and torch.equal(outs[k][1], g), k


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_high_dimensional_points(prec):
    """High-dimensional clouds (d = 16 .. 64, matrix-core passes) next to a dense
    cost in one batch: each problem's potentials are bitwise those of its own
    solve."""
    rng = np.random.default_rng(12)
    items = []
    for n, m, d, seed in ((150, 180, 32, 1), (200, 170, 64, 2), (90, 300, 16, 3)):
        p = W.embedding_problem(n, m, d, seed)
        pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
        items.append((pc, dvec(p.r), dvec(p.c)))
    C = torch.from_numpy(rng.uniform(0, 1, (100, 120)).astype(np.float32)).to(DEV)
    items.insert(1, (C, dvec(rng.dirichlet(np.ones(100))), dvec(rng.dirichlet(np.ones(120)))))
    opts = dict(gamma_init=1.0 / 8.0, gamma_final=0.02, tol=1e-6, precision=prec,
                batch_persistent=0)
    say(f"batch with high-d clouds ({prec})")
    outs, stats, status = eot.eot_solve_batched(items, workers=3, **opts)
    assert all(s == 0 for s in status)
    for k, (Ck, r, c) in enumerate(items):
        f, g, st = eot.eot_solve(Ck, r, c, **opts)
        assert torch.equal(outs[k][0], f) and torch.equal(outs[k][1], g), k
        assert stats[k]["err_r"] + stats[k]["err_c"] <= 1e-6


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cg_graph_replay_matches_direct_launches(prec):
    """CG chunks recorded once as a HIP graph and replayed give bitwise the
    potentials of direct launches: in the batch (worker streams) and for a
    single solve on a non-default stream."""
    probs, items = batch(10, seed=4300)
    kw = dict(gamma_init=1.0 / 32.0, gamma_final=1e-3, tol=1e-6, precision=prec,
              batch_persistent=0)
    say(f"cg graph batch ({prec})")
    outs0, stats0, _ = eot.eot_solve_batched(items, workers=3, **kw)
    outs1, stats1, st1 = eot.eot_solve_batched(items, workers=3, cg_graph=1, **kw)
    assert st1 == [0] * len(items)
    for k in range(len(items)):
        assert torch.equal(outs0[k][0], outs1[k][0]) and torch.equal(outs0[k][1], outs1[k][1]), k
        assert stats0[k]["cg_iters"] == stats1[k]["cg_iters"]
    pc, r, c = items[0]
    f0, g0, _ = eot.eot_solve(pc, r, c, **kw)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        f1, g1, _ = eot.eot_solve(pc, r, c, cg_graph=1, **kw)
    side.synchronize()
    assert torch.equal(f0, f1) and torch.equal(g0, g1)
