"""eot_gradient_batched (the backward over a batch of solves): every problem's
outputs against eot_gradient on it alone (with the single-launch CG off, as
the batch's host workers run it): bitwise on dense costs, to rounding on point
clouds (their gradient atomics); and one dense problem of the batch against
the oracle's derivative formulas (oracle/gradients.py, pinned by finite
differences)."""
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
    print(f"[gpu-grad-batch] {msg}", flush=True)


def dvec(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(autouse=True)
def _restore():
    yield
    eot.eot_set_cg_persist(1, 0)


def _problems():
    """Dense FP32 costs (ragged, one 3 x 7) and 2-D / 3-D point clouds, solved
    to their temperatures in FP64."""
    out = []
    for k, (n, m) in enumerate([(150, 230), (300, 210), (64, 64), (3, 7), (520, 700)]):
        rng = np.random.default_rng(40 + k)
        C = rng.uniform(0, 1, size=(n, m)).astype(np.float32)
        r = rng.dirichlet(np.ones(n)) + 1e-3; r /= r.sum()
        c = rng.dirichlet(np.ones(m)) + 1e-3; c /= c.sum()
        out.append((C, torch.from_numpy(C).to(DEV), r, c, 0.05))
    for k, (n, m, d) in enumerate([(400, 530, 2), (300, 260, 3), (129, 700, 2)]):
        p = W.point_cloud_problem(n=n, m=m, d=d, seed=90 + k)
        pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
        out.append((p, pc, p.r, p.c, 0.02))
    solved = []
    for src, Cd, r, c, gamma in out:
        f, g, _ = eot.eot_solve(Cd, dvec(r), dvec(c), gamma_init=1.0 / 8.0, gamma_final=gamma,
                                tol=1e-9, precision="fp64")
        solved.append((src, Cd, gamma, f, g))
    return solved


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("mixed", 1e-5)])
def test_gradient_batched_equals_one_by_one(prec, tol):
    probs = _problems()
    w_W, w_S = 0.6, 1.2
    say(f"batched gradient, {len(probs)} problems, {prec}")
    eot.eot_set_cg_persist(0)
    ones = [eot.eot_gradient(Cd, gamma, f, g, w_W=w_W, w_S=w_S, tol=tol, precision=prec)
            for _, Cd, gamma, f, g in probs]
    batch = eot.eot_gradient_batched([(Cd, gamma, f, g) for _, Cd, gamma, f, g in probs],
                                     w_W=w_W, w_S=w_S, tol=tol, precision=prec, workers=3)
    torch.cuda.synchronize()
    for k, (a, b) in enumerate(zip(ones, batch)):
        assert b["status"] == eot.EOT_OK
        assert b["cg_iters"] == a["cg_iters"] and b["S"] == a["S"], k
        for name in ("C", "r", "c"):
            if a.get(name) is not None:
                assert torch.equal(a[name], b[name]), (k, name)
        for name in ("X", "Y"):
            if a.get(name) is not None:
                x, y = host(a[name]), host(b[name])
                assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max(), (k, name)
    # the first problem of the batch against the oracle's formulas
    src, _, gamma, f, g = probs[0]
    u, v = O.to_log_units(host(f), host(g), gamma)
    G, gr, gc, S, _, _ = OG.vjp(src.astype(np.float64), 1.0 / gamma, u, v, w_W, w_S)
    rel = 1e-8 if prec == "fp64" else 1e-4
    assert np.abs(host(batch[0]["C"]) - G).max() <= rel * np.abs(G).max()
    assert np.abs(host(batch[0]["r"]) - gr).max() <= rel * np.abs(gr).max()
    assert abs(batch[0]["S"] - S) <= 1e-12 * S
