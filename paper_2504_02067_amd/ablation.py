"""Ablations of the solver's switches on synthetic 28 x 28 grid problems (needs a GPU).

Reproduces the shape of the paper's ablation tables (Tables 1-3) on the
blob-histogram stand-ins for MNIST: per-category pass counts (Newton/CG, line
search, ChiSinkhorn, projection), Newton steps, CG iterations and wall-clock
time, medians over seeds, for
  * the default (AdjustSchedule, warm discount rho_0, w_r = 0.45),
  * fixed decay q in {2, 4} (AdjustSchedule off),
  * rho_0 = 0 at every NewtonSolve call (warm discount off),
  * row smoothing weight w_r in {0.25, 0.35}.

    python -m paper_2504_02067_amd.ablation [--seeds 8] [--precision fp64]
"""
from __future__ import annotations

import argparse

import numpy as np
import torch

from . import eot
from . import workloads as W

VARIANTS = [
    ("default", {}),
    ("fixed q = 2", {"adaptive_q": 0, "q1": 2.0}),
    ("fixed q = 4", {"adaptive_q": 0, "q1": 4.0}),
    ("rho_0 = 0", {"adaptive_rho0": 0}),
    ("w_r = 0.35", {"w_r": 0.35}),
    ("w_r = 0.25", {"w_r": 0.25}),
]


def run(seeds=8, precision="fp64", kinds=("l1", "sqeuclid"), verbose=True):
    dev = torch.device("cuda:0")
    rows = []
    for kind in kinds:
        probs = [W.mnist_like_problem(2000 + s, kind) for s in range(seeds)]
        costs = [torch.from_numpy(p.C).to(dev) for p in probs]
        margs = [(torch.from_numpy(p.r).to(dev), torch.from_numpy(p.c).to(dev)) for p in probs]
        for name, kw in VARIANTS:
            stats = []
            for p, C, (r, c) in zip(probs, costs, margs):
                f, g, st = eot.eot_solve(C, r, c, gamma_init=p.gamma_init, gamma_final=p.gamma_final,
                                         tol=p.tol, precision=precision, allow_not_converged=True,
                                         **kw)
                stats.append(st)
            med = lambda key: float(np.median([s[key] for s in stats]))
            row = {"cost": kind, "variant": name, "seconds": med("seconds"),
                   "newton_passes": med("passes_newton"), "linesearch_passes": med("passes_linesearch"),
                   "sinkhorn_passes": med("passes_sinkhorn"), "projection_passes": med("passes_projection"),
                   "newton_steps": med("newton_steps"), "cg_iters": med("cg_iters"),
                   "mdot_steps": med("mdot_steps"),
                   "failed": sum(1 for s in stats if s["status"] != 0)}
            rows.append(row)
            if verbose:
                print(f"{kind:8s} {name:12s} {row['seconds']*1e3:8.1f} ms  NS/CG {row['newton_passes']:7.0f}  "
                      f"LS {row['linesearch_passes']:5.0f}  Sk {row['sinkhorn_passes']:5.0f}  "
                      f"proj {row['projection_passes']:5.0f}  newton {row['newton_steps']:4.0f}  "
                      f"cg {row['cg_iters']:6.0f}  mdot {row['mdot_steps']:3.0f}  failed {row['failed']}",
                      flush=True)
    return rows


def markdown(rows):
    out = ["| cost | variant | ms | NewtonSolve/CG passes | line-search passes | ChiSinkhorn passes | "
           "projection passes | Newton steps | CG iterations | MDOT steps | failed |",
           "|---|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append(f"| {r['cost']} | {r['variant']} | {r['seconds']*1e3:.1f} | {r['newton_passes']:.0f} | "
                   f"{r['linesearch_passes']:.0f} | {r['sinkhorn_passes']:.0f} | {r['projection_passes']:.0f} | "
                   f"{r['newton_steps']:.0f} | {r['cg_iters']:.0f} | {r['mdot_steps']:.0f} | {r['failed']} |")
    return "\n".join(out)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, default=8)
    ap.add_argument("--precision", default="fp64")
    a = ap.parse_args()
    print(markdown(run(a.seeds, a.precision)))
