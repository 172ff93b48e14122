"""PyTorch autograd for the entropic OT solve.

``entropic_ot(C, r, c, gamma)`` and ``entropic_ot_points(X, Y, r, c, gamma,
scale)`` return two FP64 scalars: the entropic value W (the negated dual of
Sec. 2 at the computed potentials) and the sharp transport cost S = <P, C>.
Their backward is one ``eot_gradient`` call of the C ABI, which receives the
upstream gradients of W and S as weights (a vector-Jacobian product): W
differentiates by the envelope theorem, S by implicit differentiation of the
marginal constraints through the dual Hessian, solved with the CG of Alg. 2
at rho = 1. Gradients for r and c have their mean removed (r and c live on
the simplex). This module only marshals tensors; every step runs in the HIP
library.
"""
from __future__ import annotations

import torch

from . import eot


def _split(kw):
    """Solve options, and the backward's (tol, max_cg, precision) passed with a
    ``grad_`` prefix."""
    solve = {k: v for k, v in kw.items() if not k.startswith("grad_")}
    grad = {k[5:]: v for k, v in kw.items() if k.startswith("grad_")}
    return solve, grad, solve.pop("precision", "fp64")


class _EntropicOT(torch.autograd.Function):
    @staticmethod
    def forward(ctx, C, X, Y, r, c, gamma, scale, kw):
        if C is not None:
            cost = C.detach()
        else:
            cost = eot.PointCloud(X.detach().contiguous(), Y.detach().contiguous(), scale)
        solve_kw, grad_kw, prec = _split(dict(kw))
        solve_kw.setdefault("gamma_init", max(gamma, 1.0 / 32.0))
        f, g, st = eot.eot_solve(cost, r.detach().double().contiguous(),
                                 c.detach().double().contiguous(), gamma_final=gamma,
                                 precision=prec, **solve_kw)
        ctx.cost = cost
        ctx.gamma = gamma
        ctx.grad_kw = grad_kw
        ctx.shapes = (C is not None, X.dtype if X is not None else None,
                      C.dtype if C is not None else None, r.dtype, c.dtype)
        ctx.save_for_backward(f, g)
        ctx.stats = st
        dev = r.device
        W = torch.tensor(st["dual_value"], dtype=torch.float64, device=dev)
        S = torch.tensor(st["cost"], dtype=torch.float64, device=dev)
        return W, S

    @staticmethod
    def backward(ctx, gW, gS):
        f, g = ctx.saved_tensors
        dense, xdt, cdt, rdt, cdt2 = ctx.shapes
        need = ctx.needs_input_grad
        want = []
        if dense and need[0]:
            want.append("C")
        if not dense and need[1]:
            want.append("X")
        if not dense and need[2]:
            want.append("Y")
        if need[3]:
            want.append("r")
        if need[4]:
            want.append("c")
        wW = 0.0 if gW is None else float(gW)
        wS = 0.0 if gS is None else float(gS)
        out = eot.eot_gradient(ctx.cost, ctx.gamma, f, g, w_W=wW, w_S=wS, want=tuple(want),
                               **ctx.grad_kw)
        gC = out["C"].to(cdt) if out["C"] is not None else None
        gX = out["X"].to(xdt) if out["X"] is not None else None
        gY = out["Y"].to(xdt) if out["Y"] is not None else None
        gr = out["r"].to(rdt) if out["r"] is not None else None
        gc = out["c"].to(cdt2) if out["c"] is not None else None
        return gC, gX, gY, gr, gc, None, None, None


def entropic_ot(C: torch.Tensor, r: torch.Tensor, c: torch.Tensor, gamma: float, **kw):
    """(W, S) for a dense cost C (float32 / float64 GPU tensor, n x m) at
    temperature gamma. Keyword arguments go to the solve (gamma_init, tol,
    precision, ...) or, as tol/max_cg prefixed with ``grad_``, to the
    backward's CG."""
    return _EntropicOT.apply(C, None, None, r, c, float(gamma), 1.0, tuple(kw.items()))


def entropic_ot_points(X: torch.Tensor, Y: torch.Tensor, r: torch.Tensor, c: torch.Tensor,
                       gamma: float, scale: float, **kw):
    """(W, S) for the point-cloud cost C_ij = |x_i - y_j|^2 / scale (X: n x d,
    Y: m x d float32 GPU tensors, d in {2, 3, 16, 32, 48, 64}), recomputed on the
    fly."""
    return _EntropicOT.apply(None, X, Y, r, c, float(gamma), float(scale), tuple(kw.items()))
