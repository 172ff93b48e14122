"""GPU parity of eot_hvp_with_marginals: the discounted Hessian-vector product
of eqs. hessian / discounted-hessian with the diagonal blocks D(r(P)), D(c(P))
taken from given log marginals, against the FP64 oracle's HVP (which forms
r(P) and c(P) itself), for dense costs, 2-D / 3-D point clouds and
high-dimensional clouds, ragged shapes included.

The marginals passed in are the oracle's (exact to FP64 rounding), so the
tolerances are those of eot_hvp: 1e-12 relative to the absolute-value product
in FP64, the mixed bound of each cost kind in mixed precision. With the
library's own mixed marginals (the full-size sampled test of the point-cloud
file) the diagonal carries the mixed error of the marginals, within the same
bound."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2504_02067_amd import eot
from paper_2504_02067_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def say(msg):
    print(f"[gpu-hvp-marg] {msg}", flush=True)


def dvec(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def check(C, Cd, gamma, u, v, rho, prec, tol, seed):
    """Both outputs against the oracle, and against eot_hvp on the same input."""
    n, m = C.shape
    beta = 1.0 / gamma
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n); y = rng.standard_normal(m)
    f, g = u * gamma, v * gamma
    uu, vv = O.to_log_units(f, g, gamma)
    lr = O.log_row_marginal(C, beta, uu, vv)
    lc = O.log_col_marginal(C, beta, uu, vv)
    Hx, Hy = eot.eot_hvp_with_marginals(Cd, gamma, dvec(f), dvec(g), dvec(lr), dvec(lc), rho,
                                        dvec(x), dvec(y), precision=prec)
    Fx, Fy = eot.eot_hvp(Cd, gamma, dvec(f), dvec(g), rho, dvec(x), dvec(y), precision=prec)
    torch.cuda.synchronize()
    Hx_ref, Hy_ref = O.hvp(C, beta, uu, vv, rho, x, y)
    ax, ay = O.hvp(C, beta, uu, vv, rho, np.abs(x), np.abs(y))
    assert np.all(np.abs(host(Hx) - Hx_ref) <= tol * ax + 1e-300)
    assert np.all(np.abs(host(Hy) - Hy_ref) <= tol * ay + 1e-300)
    assert np.all(np.abs(host(Hx) - host(Fx)) <= 2 * tol * ax + 1e-300)
    assert np.all(np.abs(host(Hy) - host(Fy)) <= 2 * tol * ay + 1e-300)


@pytest.mark.parametrize("n,m,cdt", [(300, 4500, np.float32), (130, 2049, np.float32),
                                     (64, 64, np.float64), (1, 5, np.float32),
                                     (7, 1, np.float32)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("rho", [1.0, 0.5625, 0.0])
def test_dense_hvp_with_marginals(n, m, cdt, prec, rho):
    gamma = 0.05
    if prec == "mixed" and cdt == np.float64:
        # mixed precision reads an FP32 cost: the library rejects an FP64 one
        z = lambda k: torch.zeros(k, dtype=torch.float64, device=DEV)  # noqa: E731
        with pytest.raises(eot.EotError) as e:
            eot.eot_hvp_with_marginals(torch.zeros(n, m, dtype=torch.float64, device=DEV), gamma,
                                       z(n), z(m), z(n), z(m), rho, z(n), z(m), precision=prec)
        assert e.value.status == eot.EOT_ERR_UNSUPPORTED
        return
    rng = np.random.default_rng(n + 7 * m)
    C = rng.uniform(0.0, 1.0, size=(n, m)).astype(cdt)
    u = np.log(rng.dirichlet(np.ones(n))) + rng.standard_normal(n)
    v = np.log(rng.dirichlet(np.ones(m))) + rng.standard_normal(m)
    say(f"dense n={n} m={m} {cdt.__name__} {prec} rho={rho}")
    check(C.astype(np.float64), torch.from_numpy(C).to(DEV), gamma, u, v, rho, prec,
          1e-12 if prec == "fp64" else 4e-6, n + m)


@pytest.mark.parametrize("n,m,d", [(700, 2100, 3), (257, 256, 2), (1, 5, 3), (130, 2049, 3)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("rho", [1.0, 0.5])
def test_points_hvp_with_marginals(n, m, d, prec, rho):
    gamma = 0.05
    beta = 1.0 / gamma
    rng = np.random.default_rng(n + m + d)
    X = W.gmm_points(rng, n, d=d); Y = W.gmm_points(rng, m, d=d)
    s = W.bbox_scale(X, Y)
    pc = eot.PointCloud(torch.from_numpy(X).to(DEV), torch.from_numpy(Y).to(DEV), s)
    C = O.sqeuclid_points_cost(X, Y, s)
    u = -np.log(n) + rng.standard_normal(n)
    v = -np.log(m) - O.log_col_marginal(C, beta, u, np.zeros(m))
    say(f"points n={n} m={m} d={d} {prec} rho={rho}")
    check(C, pc, gamma, u, v, rho, prec, 1e-12 if prec == "fp64" else 4e-6 + 3e-7 * beta * C.max(),
          d)


@pytest.mark.parametrize("d,n,m", [(16, 130, 517), (64, 333, 1100)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_highd_hvp_with_marginals(d, n, m, prec):
    gamma, rho = 0.05, 0.5
    beta = 1.0 / gamma
    p = W.embedding_problem(n, m, d, 3 + d)
    pc = eot.PointCloud(torch.from_numpy(p.X).to(DEV), torch.from_numpy(p.Y).to(DEV), p.scale)
    C = O.sqeuclid_points_cost(p.X, p.Y, p.scale)
    rng = np.random.default_rng(5)
    u = np.log(p.r) + 0.5 * rng.standard_normal(n)
    v = np.log(p.c) - O.log_col_marginal(C, beta, u, np.zeros(m))
    say(f"high-d d={d} n={n} m={m} {prec}")
    check(C, pc, gamma, u, v, rho, prec, 1e-12 if prec == "fp64" else 4e-6 + 1.2e-5 * beta, d)


def test_hvp_with_marginals_rejects_bad_rho():
    C = torch.rand(8, 8, device=DEV, dtype=torch.float32)
    z8 = torch.zeros(8, dtype=torch.float64, device=DEV)
    with pytest.raises(eot.EotError) as e:
        eot.eot_hvp_with_marginals(C, 0.1, z8, z8, z8, z8, 1.5, z8, z8)
    assert e.value.status == eot.EOT_ERR_INVALID_ARG
