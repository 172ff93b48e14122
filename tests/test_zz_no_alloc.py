"""eot_hvp_noalloc (the entry point that allocates nothing and runs on the
library's own per-GPU scratch) against eot_hvp (caller workspace) through the
C ABI: two calls in a row, the second on a smaller problem, so the second
call runs on scratch that still holds the first call's contents. Both entry
points run the same kernels in the same order, so the outputs must agree
bitwise."""
import numpy as np
import pytest
import torch

from paper_2504_02067_amd import eot

pytestmark = pytest.mark.gpu


def _dense(rng, n, m, dtype):
    C = rng.uniform(0.0, 1.0, (n, m)).astype(dtype)
    return torch.from_numpy(C).cuda()


def _points(rng, n, m, d):
    X = torch.from_numpy(rng.uniform(-1, 1, (n, d)).astype(np.float32)).cuda()
    Y = torch.from_numpy(rng.uniform(-1, 1, (m, d)).astype(np.float32)).cuda()
    return eot.PointCloud(X, Y, 4.0 * d)


def _case(rng, C, n, m, gamma, rho, prec):
    f = torch.from_numpy(gamma * (np.log(1.0 / n) + 0.3 * rng.standard_normal(n))).cuda()
    g = torch.from_numpy(gamma * (np.log(1.0 / m) + 0.3 * rng.standard_normal(m))).cuda()
    x = torch.from_numpy(rng.standard_normal(n)).cuda()
    y = torch.from_numpy(rng.standard_normal(m)).cuda()
    want = eot.eot_hvp(C, gamma, f, g, rho, x, y, precision=prec)
    got = eot.eot_hvp_noalloc(C, gamma, f, g, rho, x, y, precision=prec)
    torch.cuda.synchronize()
    return want, got


@pytest.mark.parametrize("kind,prec", [("f32", "mixed"), ("f32", "fp64"), ("f64", "fp64"),
                                       ("points3", "mixed"), ("points64", "mixed")])
def test_noalloc_hvp_equals_workspace_hvp_twice(kind, prec):
    rng = np.random.default_rng(11)
    # first call larger (several 2048-column tiles, ragged rows), second smaller
    for (n, m) in ((5000, 4500), (700, 333)):
        print(f"[no_alloc] {kind} {prec} n={n} m={m}", flush=True)
        if kind == "f32":
            C = _dense(rng, n, m, np.float32)
        elif kind == "f64":
            C = _dense(rng, n, m, np.float64)
        else:
            C = _points(rng, n, m, 3 if kind == "points3" else 64)
        (hx, hy), (gx, gy) = _case(rng, C, n, m, 0.05, 0.5625, prec)
        assert torch.isfinite(hx).all() and torch.isfinite(hy).all()
        assert torch.equal(hx, gx) and torch.equal(hy, gy), (
            (hx - gx).abs().max().item(), (hy - gy).abs().max().item())


def test_noalloc_rejects_oversize_before_device_work():
    import ctypes
    big = eot.eot_cost(kind=0, d=0, n=32768, m=32768, ldc=32768, C=ctypes.c_void_p(4096),
                       X=None, Y=None, scale=0.0)
    p = ctypes.c_void_p(8)
    st = eot.lib().eot_hvp_noalloc(ctypes.byref(big), 0.1, p, p, None, 0.5, p, p, p, p, 1,
                                   None)
    assert st == eot.EOT_ERR_WORKSPACE
