"""Derivatives of the entropic OT value and of the sharp transport cost, in
plain dense FP64 NumPy (TEST INFRASTRUCTURE ONLY, like the rest of oracle/).

Notation (log units, Sec. 2): P_ij = exp(u_i + v_j - beta C_ij), r(P) = P 1,
c(P) = P^T 1, temperature gamma = 1 / beta, cost-unit potentials f = u / beta,
g = v / beta. The value is the dual objective at the potentials,

    W = gamma (<u, r> + <v, c> - sum_ij P_ij + 1),

which at the optimum equals the entropic primal, and the sharp cost is
S = <P, C>.

* W: by the envelope theorem dW/dC = P, dW/dr = f, dW/dc = g.
* S: the optimality conditions r(P) = r, c(P) = c define (u, v) implicitly;
  their differential is H [du; dv] = [dr; dc] + beta [(P o dC) 1; (P o dC)^T 1]
  with H the dual Hessian [[D(r(P)), P], [P^T, D(c(P))]] (Sec. 2, Hessian of
  the dual). With [lam; mu] = H^+ [(P o C) 1; (P o C)^T 1] this gives
  dS/dC_ij = P_ij (1 + beta (lam_i + mu_j - C_ij)), dS/dr = lam, dS/dc = mu.
* Point clouds, C_ij = |x_i - y_j|^2 / s: dC_ij/dx_i = 2 (x_i - y_j) / s, so
  d/dX = (2/s) (X o (G 1) - G Y) and d/dY = (2/s) (Y o (G^T 1) - G^T X) for
  any cotangent G of C.

Gradients with respect to r and c are returned with their mean removed (the
component along the simplex's tangent space; the constant part is not defined
because r and c are constrained to sum to one).
"""
from __future__ import annotations

import numpy as np


def plan(C, beta, u, v):
    C = np.asarray(C, dtype=np.float64)
    return np.exp(np.asarray(u)[:, None] + np.asarray(v)[None, :] - beta * C)


def value(C, beta, u, v, r, c):
    """W = gamma (<u, r> + <v, c> - sum P + 1) in cost units."""
    P = plan(C, beta, u, v)
    return (np.dot(u, r) + np.dot(v, c) - P.sum() + 1.0) / beta


def hessian_solve(P, a, b):
    """Minimum-norm solution of [[D(P 1), P], [P^T, D(P^T 1)]] [lam; mu] = [a; b]
    (dense least squares; H is singular along (1, -1))."""
    n, m = P.shape
    H = np.zeros((n + m, n + m))
    H[:n, :n] = np.diag(P.sum(1))
    H[n:, n:] = np.diag(P.sum(0))
    H[:n, n:] = P
    H[n:, :n] = P.T
    sol = np.linalg.lstsq(H, np.concatenate([a, b]), rcond=1e-14)[0]
    return sol[:n], sol[n:]


def _centre(x):
    return x - x.mean()


def vjp(C, beta, u, v, w_W, w_S):
    """Cotangent of C and gradients for r, c of w_W W + w_S S at (u, v).

    Returns (G, grad_r, grad_c, S, lam, mu): G_ij = w_W P_ij + w_S P_ij
    (1 + beta (lam_i + mu_j - C_ij)); grad_r = w_W f + w_S lam and grad_c =
    w_W g + w_S mu, mean removed."""
    C = np.asarray(C, dtype=np.float64)
    P = plan(C, beta, u, v)
    PC = P * C
    S = PC.sum()
    n, m = P.shape
    lam, mu = np.zeros(n), np.zeros(m)
    if w_S != 0.0:
        lam, mu = hessian_solve(P, PC.sum(1), PC.sum(0))
    G = w_W * P + w_S * P * (1.0 + beta * (lam[:, None] + mu[None, :] - C))
    f, g = np.asarray(u) / beta, np.asarray(v) / beta
    return G, _centre(w_W * f + w_S * lam), _centre(w_W * g + w_S * mu), S, lam, mu


def points_grad(X, Y, scale, G):
    """(dL/dX, dL/dY) for a cotangent G of C = |x - y|^2 / scale."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    gX = (2.0 / scale) * (X * G.sum(1)[:, None] - G @ Y)
    gY = (2.0 / scale) * (Y * G.sum(0)[:, None] - G.T @ X)
    return gX, gY
