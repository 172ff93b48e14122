"""Seeded synthetic OT instances.

This module only builds problem data (costs, marginals, point clouds). It
holds none of the solver's arithmetic, so both the HIP path and the FP64
oracle can be fed from it.

The paper's datasets (upsampled MNIST, colour-transfer images, DOTmark) are
not available; the instances below stand in for them with the same shapes,
value ranges and structure:

* squared-Euclidean costs between uniform random points, Dirichlet
  marginals (small FP64 problem);
* histograms on square pixel grids made of a few Gaussian blobs with
  near-zero background (the image histograms of Sec. 4.1 / App. E), with
  L1 or squared-L2 grid-distance costs normalised to max 1 (Sec. 2.1 asks
  for C in [0, 1]);
* Gaussian-mixture point clouds in R^3 with uniform marginals (the RGB
  colour-transfer problem of Sec. 4.1 and Fig. 3).

Every generator draws from ``numpy.random.default_rng(seed)`` in a fixed
order: points first, then the row-marginal blobs, then the column-marginal
blobs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Problem:
    """One OT instance. ``C`` is row-major (n, m); ``X``/``Y`` are set for
    point-cloud costs, where C = |x - y|^2 / scale."""
    name: str
    n: int
    m: int
    r: np.ndarray                      # float64 (n,), sums to 1
    c: np.ndarray                      # float64 (m,), sums to 1
    C: Optional[np.ndarray] = None     # float32 or float64 (n, m)
    X: Optional[np.ndarray] = None     # float32 (n, d)
    Y: Optional[np.ndarray] = None     # float32 (m, d)
    scale: float = 1.0                 # point-cloud cost normaliser
    gamma_init: float = 1.0 / 32.0     # temperatures (1/gamma_paper)
    gamma_final: float = 1e-3
    tol: float = 1e-6
    meta: dict = field(default_factory=dict)


# ---------------------------------------------------------------- marginals

def _normalise(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    return x / x.sum()


def dirichlet_marginal(rng: np.random.Generator, n: int, floor: float = 1e-6) -> np.ndarray:
    """Dirichlet(1) draw plus a floor, renormalised."""
    w = rng.dirichlet(np.ones(n))
    return _normalise(w + floor)


def blob_histogram(rng: np.random.Generator, side: int, nblobs: int = 3,
                   sigma_lo: float = 1.5, sigma_hi: float = 4.0,
                   cut: float = 0.01, floor: float = 1e-6) -> np.ndarray:
    """Sum of isotropic Gaussian blobs with unit peak on a side x side grid.

    Centres ~ U[0, side-1]^2, sigma ~ U[sigma_lo, sigma_hi] pixels; pixels
    below ``cut`` times the maximum are zeroed (the near-zero background of
    image histograms), then ``floor`` is added and the result normalised.
    Flattened in row-major pixel order (index = y * side + x).
    """
    ys, xs = np.mgrid[0:side, 0:side].astype(np.float64)
    h = np.zeros((side, side), dtype=np.float64)
    for _ in range(nblobs):
        cy, cx = rng.uniform(0.0, side - 1, size=2)
        s = rng.uniform(sigma_lo, sigma_hi)
        h += np.exp(-((ys - cy) ** 2 + (xs - cx) ** 2) / (2.0 * s * s))
    h[h < cut * h.max()] = 0.0
    return _normalise(h.reshape(-1) + floor)


# -------------------------------------------------------------------- costs

def grid_coords(side: int) -> np.ndarray:
    """(side*side, 2) integer pixel coordinates (y, x), row-major order."""
    ys, xs = np.mgrid[0:side, 0:side]
    return np.stack([ys.reshape(-1), xs.reshape(-1)], axis=1).astype(np.int64)


def grid_cost(side: int, kind: str = "sqeuclid", dtype=np.float32) -> np.ndarray:
    """Pairwise L1 or squared-L2 pixel distance divided by its maximum.

    Distances are integers, computed exactly; the one division by the max is
    done in ``dtype`` (correctly rounded), so the matrix is reproducible.
    """
    p = grid_coords(side)
    dy = np.abs(p[:, None, 0] - p[None, :, 0])
    dx = np.abs(p[:, None, 1] - p[None, :, 1])
    if kind == "sqeuclid":
        d = dy * dy + dx * dx
    elif kind == "l1":
        d = dy + dx
    else:
        raise ValueError(kind)
    d = d.astype(dtype)
    return d / dtype(d.max())


def grid_cost_rows(side: int, rows: np.ndarray, kind: str = "sqeuclid",
                   dtype=np.float32) -> np.ndarray:
    """Selected rows of :func:`grid_cost` without building the full matrix."""
    p = grid_coords(side)
    q = p[np.asarray(rows)]
    dy = np.abs(q[:, None, 0] - p[None, :, 0])
    dx = np.abs(q[:, None, 1] - p[None, :, 1])
    if kind == "sqeuclid":
        d = dy * dy + dx * dx
        dmax = 2 * (side - 1) ** 2
    else:
        d = dy + dx
        dmax = 2 * (side - 1)
    return d.astype(dtype) / dtype(dmax)


def sqeuclid_cost(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """|x_i - y_j|^2 / max, in float64, difference form."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    d = ((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    return d / d.max()


# ---------------------------------------------------------------- instances

def small_points_problem(seed: int = 1000, n: int = 64) -> Problem:
    """n = m = 64 uniform points in [0,1]^2, Dirichlet(1) marginals with a
    1e-6 floor, FP64 cost; temperature annealed 1e-1 -> 1e-3, tol 1e-9."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, size=(n, 2))
    Y = rng.uniform(0.0, 1.0, size=(n, 2))
    r = dirichlet_marginal(rng, n)
    c = dirichlet_marginal(rng, n)
    C = sqeuclid_cost(X, Y)
    return Problem(name=f"points64_s{seed}", n=n, m=n, r=r, c=c, C=C,
                   gamma_init=1e-1, gamma_final=1e-3, tol=1e-9,
                   meta={"seed": seed, "cost": "sqeuclid", "dtype": "f64"})


def grid_blob_problem(side: int, seed: int, kind: str = "sqeuclid",
                      gamma_final: float = 1e-4, tol: float = 1e-6,
                      build_cost: bool = True) -> Problem:
    """side x side grid, 3-blob histograms, L1 / squared-L2 cost in FP32."""
    rng = np.random.default_rng(seed)
    r = blob_histogram(rng, side)
    c = blob_histogram(rng, side)
    n = side * side
    C = grid_cost(side, kind) if build_cost else None
    return Problem(name=f"grid{side}_{kind}_s{seed}", n=n, m=n, r=r, c=c, C=C,
                   gamma_init=1.0 / 32.0, gamma_final=gamma_final, tol=tol,
                   meta={"seed": seed, "side": side, "cost": kind, "dtype": "f32"})


def mnist_like_problem(seed: int = 2000, kind: str = "sqeuclid") -> Problem:
    """n = m = 784 (28 x 28 grid), annealed to temperature 1e-4."""
    return grid_blob_problem(28, seed, kind, gamma_final=1e-4, tol=1e-6)


def large_grid_problem(seed: int = 3000, build_cost: bool = False) -> Problem:
    """n = m = 16384 (128 x 128 grid), squared-L2, annealed to 1e-5.

    The dense FP32 cost is 1 GiB; by default it is not built on the host
    (use :func:`grid_cost_rows` for samples, or build it on the device)."""
    return grid_blob_problem(128, seed, "sqeuclid", gamma_final=1e-5, tol=1e-6,
                             build_cost=build_cost)


def batch_sides(seed: int = 4000, count: int = 512, lo: int = 16, hi: int = 64) -> np.ndarray:
    """Grid side lengths of the ragged batch, uniform on {lo..hi}."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=count)


def batch_problem(index: int, seed: int = 4000, sides: Optional[np.ndarray] = None) -> Problem:
    """Problem ``index`` of the 512-problem ragged batch (temperature 1e-3).

    Points are the integer grid positions as FP32 (d = 2) and the cost is
    |x - y|^2 / (2 (side - 1)^2)."""
    if sides is None:
        sides = batch_sides(seed)
    side = int(sides[index])
    p = grid_blob_problem(side, seed * 1000 + index, "sqeuclid",
                          gamma_final=1e-3, tol=1e-6)
    X = grid_coords(side).astype(np.float32)
    p.X = X
    p.Y = X.copy()
    p.scale = float(2 * (side - 1) ** 2)
    p.name = f"batch{index}_side{side}"
    return p


def gmm_points(rng: np.random.Generator, n: int, k: int = 8, d: int = 3) -> np.ndarray:
    """n points from a k-component isotropic GMM: means ~ U[-1,1]^d,
    sigma ~ U[0.05, 0.2], equal weights."""
    means = rng.uniform(-1.0, 1.0, size=(k, d))
    sig = rng.uniform(0.05, 0.2, size=k)
    comp = rng.integers(0, k, size=n)
    pts = means[comp] + sig[comp, None] * rng.standard_normal((n, d))
    return pts.astype(np.float32)


def bbox_scale(X: np.ndarray, Y: np.ndarray) -> float:
    """Squared diagonal of the box holding both clouds: an upper bound of every
    |x - y|^2, so C = |x - y|^2 / scale lies in [0, 1] (the exact maximum
    would cost an n x m sweep)."""
    Z = np.concatenate([np.asarray(X, np.float64), np.asarray(Y, np.float64)])
    ext = Z.max(0) - Z.min(0)
    return float((ext * ext).sum())


def point_cloud_problem(n: int = 1 << 20, seed: int = 5000, m: Optional[int] = None,
                        d: int = 3) -> Problem:
    """Two 8-component Gaussian mixtures in R^d (m points in the second),
    uniform marginals, cost recomputed on the fly as |x - y|^2 / s with s the
    squared bounding-box diagonal (:func:`bbox_scale`)."""
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    X = gmm_points(rng, n, d=d)
    Y = gmm_points(rng, m, d=d)
    r = np.full(n, 1.0 / n)
    c = np.full(m, 1.0 / m)
    return Problem(name=f"gmm{d}d_n{n}_m{m}_s{seed}", n=n, m=m, r=r, c=c, X=X, Y=Y,
                   scale=bbox_scale(X, Y), gamma_init=1.0 / 32.0, gamma_final=1e-4,
                   tol=1e-4, meta={"seed": seed, "cost": "sqeuclid_points", "d": d})


def embedding_points(rng: np.random.Generator, n: int, d: int, k: int = 8,
                     spread: float = 0.5) -> np.ndarray:
    """n unit vectors in R^d around k random unit directions (normalised
    direction + spread * N(0, I / d)), FP32."""
    mu = rng.standard_normal((k, d))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    comp = rng.integers(0, k, size=n)
    P = mu[comp] + spread * rng.standard_normal((n, d)) / np.sqrt(d)
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    return P.astype(np.float32)


def embedding_problem(n: int = 1 << 16, m: Optional[int] = None, d: int = 64,
                      seed: int = 6000) -> Problem:
    """Two clouds of unit-norm embeddings in R^d (8 shared directions),
    uniform marginals, cost |x - y|^2 / 4 (4 bounds the squared distance of
    unit vectors), recomputed on the fly."""
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    X = embedding_points(rng, n, d)
    Y = embedding_points(rng, m, d)
    return Problem(name=f"emb{d}d_n{n}_m{m}_s{seed}", n=n, m=m, r=np.full(n, 1.0 / n),
                   c=np.full(m, 1.0 / m), X=X, Y=Y, scale=4.0, gamma_init=1.0 / 8.0,
                   gamma_final=1e-2, tol=1e-5,
                   meta={"seed": seed, "cost": "sqeuclid_points", "d": d})


def random_potentials(rng: np.random.Generator, n: int, m: int, gamma: float,
                      spread: float = 1.0):
    """Potentials in cost units for kernel-level tests: f, g ~ spread * N(0,1)
    minus a constant that keeps the plan mass near 1 for costs in [0, 1]."""
    f = spread * gamma * rng.standard_normal(n)
    g = spread * gamma * rng.standard_normal(m)
    return f, g


def grid_cost_device(side: int, kind: str = "sqeuclid", device="cuda", block: int = 2048):
    """:func:`grid_cost` built directly in device memory as float32 (same
    integer distances and the same single float32 division by the max), in
    row blocks so no n x n integer temporary is materialised."""
    import torch
    n = side * side
    idx = torch.arange(n, device=device)
    py, px = idx // side, idx % side
    dmax = 2 * (side - 1) ** 2 if kind == "sqeuclid" else 2 * (side - 1)
    out = torch.empty((n, n), dtype=torch.float32, device=device)
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        dy = (py[i0:i1, None] - py[None, :]).abs()
        dx = (px[i0:i1, None] - px[None, :]).abs()
        d = dy * dy + dx * dx if kind == "sqeuclid" else dy + dx
        out[i0:i1] = d.to(torch.float32) / torch.tensor(float(dmax), dtype=torch.float32,
                                                       device=device)
    return out
