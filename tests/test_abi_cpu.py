"""CPU checks of the C ABI library: it loads, exports every entry point that
include/eot.h declares, and its host-only logic (workspace sizing, argument
validation, status strings, option defaults) behaves as documented. No
kernel is launched."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eot.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eot_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2504_02067_amd import eot
    if not os.path.exists(eot.LIB_PATH):
        pytest.fail("libeot.so not built (run __graft_entry__.build())")
    return eot.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("eot_marginals", "eot_hvp", "eot_hvp_with_marginals", "eot_newton_cg", "eot_solve",
              "eot_workspace_size",
              "eot_status_string", "eot_version", "eot_solve_opts_default"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    from paper_2504_02067_amd import eot
    for name in _declared():
        assert hasattr(L, name), name
        assert name in eot.SIGNATURES, f"binding lacks {name}"


def test_status_strings_and_version(L):
    from paper_2504_02067_amd import eot
    assert eot.version().endswith("gfx950")
    seen = set()
    for s in range(8):
        txt = eot.status_string(s)
        assert txt and txt != "unknown status"
        seen.add(txt)
    assert len(seen) == 8
    assert eot.status_string(99) == "unknown status"


def test_workspace_size_scales_and_validates(L):
    from paper_2504_02067_amd import eot
    sz = ctypes.c_size_t(0)

    def ws(op, n, m, kind=0):
        c = eot.eot_cost(kind=kind, d=0, n=n, m=m, ldc=m, C=ctypes.c_void_p(4096), X=None,
                         Y=None, scale=0.0)
        st = L.eot_workspace_size(op, ctypes.byref(c), 0, ctypes.byref(sz))
        return st, sz.value

    st, small = ws(eot.EOT_OP_SOLVE, 64, 64)
    assert st == eot.EOT_OK and small > 0
    st, big = ws(eot.EOT_OP_SOLVE, 16384, 16384)
    assert st == eot.EOT_OK and big > 100 * small
    for op in range(5):
        assert ws(op, 1, 1)[0] == eot.EOT_OK
    assert ws(eot.EOT_OP_SOLVE, 0, 5)[0] == eot.EOT_ERR_INVALID_ARG
    assert ws(7, 5, 5)[0] == eot.EOT_ERR_INVALID_ARG
    assert ws(0, 5, 5, kind=9)[0] == eot.EOT_ERR_INVALID_ARG
    assert L.eot_workspace_size(0, None, 0, ctypes.byref(sz)) == eot.EOT_ERR_INVALID_ARG


def test_argument_validation_happens_before_any_device_work(L):
    from paper_2504_02067_amd import eot
    c = eot.eot_cost(kind=0, d=0, n=8, m=8, ldc=8, C=ctypes.c_void_p(4096), X=None, Y=None,
                     scale=0.0)
    p = ctypes.c_void_p(4096)
    # bad temperature, null potentials, null outputs
    assert L.eot_marginals(ctypes.byref(c), -1.0, p, p, None, p, None, None, None, None, 0,
                           p, 1 << 20, None) == eot.EOT_ERR_INVALID_ARG
    assert L.eot_marginals(ctypes.byref(c), float("nan"), p, p, None, p, None, None, None, None,
                           0, p, 1 << 20, None) == eot.EOT_ERR_INVALID_ARG
    assert L.eot_marginals(ctypes.byref(c), 1.0, None, p, None, p, None, None, None, None, 0,
                           p, 1 << 20, None) == eot.EOT_ERR_INVALID_ARG
    assert L.eot_marginals(ctypes.byref(c), 1.0, p, p, None, None, None, None, None, None, 0,
                           p, 1 << 20, None) == eot.EOT_ERR_INVALID_ARG
    # s requested without c_for_s
    assert L.eot_marginals(ctypes.byref(c), 1.0, p, p, None, p, None, None, None, p, 0,
                           p, 1 << 20, None) == eot.EOT_ERR_INVALID_ARG
    # rho outside [0, 1]
    assert L.eot_hvp(ctypes.byref(c), 1.0, p, p, None, 1.5, p, p, p, p, 0, p, 1 << 20,
                     None) == eot.EOT_ERR_INVALID_ARG
    # the HVP with the marginals given: both marginals required, rho in [0, 1], gamma > 0
    hm = L.eot_hvp_with_marginals
    assert hm(ctypes.byref(c), 1.0, p, p, None, p, 1.0, p, p, p, p, 0, p, 1 << 20,
              None) == eot.EOT_ERR_INVALID_ARG
    assert hm(ctypes.byref(c), 1.0, p, p, p, None, 1.0, p, p, p, p, 0, p, 1 << 20,
              None) == eot.EOT_ERR_INVALID_ARG
    assert hm(ctypes.byref(c), 1.0, p, p, p, p, -0.5, p, p, p, p, 0, p, 1 << 20,
              None) == eot.EOT_ERR_INVALID_ARG
    assert hm(ctypes.byref(c), 0.0, p, p, p, p, 1.0, p, p, p, p, 0, p, 1 << 20,
              None) == eot.EOT_ERR_INVALID_ARG
    assert hm(ctypes.byref(c), 1.0, p, p, p, p, 1.0, p, p, None, p, 0, p, 1 << 20,
              None) == eot.EOT_ERR_INVALID_ARG
    assert hm(ctypes.byref(c), 1.0, p, p, p, p, 1.0, p, p, p, p, 0, p, 16,
              None) == eot.EOT_ERR_WORKSPACE
    # mixed precision on an FP64 dense cost is not supported
    c64 = eot.eot_cost(kind=1, d=0, n=8, m=8, ldc=8, C=ctypes.c_void_p(4096), X=None, Y=None,
                       scale=0.0)
    assert hm(ctypes.byref(c64), 1.0, p, p, p, p, 1.0, p, p, p, p, 1, p, 1 << 20,
              None) == eot.EOT_ERR_UNSUPPORTED
    assert L.eot_marginals(ctypes.byref(c64), 1.0, p, p, None, p, None, None, None, None, 1,
                           p, 1 << 20, None) == eot.EOT_ERR_UNSUPPORTED
    # workspace too small / misaligned
    assert L.eot_marginals(ctypes.byref(c), 1.0, p, p, None, p, None, None, None, None, 0,
                           p, 16, None) == eot.EOT_ERR_WORKSPACE
    assert L.eot_marginals(ctypes.byref(c), 1.0, p, p, None, p, None, None, None, None, 0,
                           ctypes.c_void_p(4100), 1 << 20, None) == eot.EOT_ERR_WORKSPACE
    # ldc < m
    bad = eot.eot_cost(kind=0, d=0, n=8, m=8, ldc=4, C=p, X=None, Y=None, scale=0.0)
    assert L.eot_marginals(ctypes.byref(bad), 1.0, p, p, None, p, None, None, None, None, 0,
                           p, 1 << 20, None) == eot.EOT_ERR_INVALID_ARG
    # solve options
    o = eot.eot_solve_opts()
    L.eot_solve_opts_default(ctypes.byref(o))
    assert (o.p, o.q1, o.w_r, o.adaptive_q, o.adaptive_rho0) == (1.5, 2.0, 0.45, 1, 1)
    assert o.max_backtrack == 60 and o.verify_fp64 == 1
    assert o.cg_graph == 0 and o.verbose == 0
    o.w_r = 0.6
    st = eot.eot_solve_stats()
    assert L.eot_solve(ctypes.byref(c), p, p, ctypes.byref(o), p, p, ctypes.byref(st), p,
                       1 << 20, None) == eot.EOT_ERR_INVALID_ARG
    o.w_r = 0.45
    o.gamma_final = 0.0
    assert L.eot_solve(ctypes.byref(c), p, p, ctypes.byref(o), p, p, ctypes.byref(st), p,
                       1 << 20, None) == eot.EOT_ERR_INVALID_ARG


def test_gradient_and_points_validation(L):
    from paper_2504_02067_amd import eot
    p = ctypes.c_void_p(4096)
    dense = eot.eot_cost(kind=0, d=0, n=8, m=8, ldc=8, C=p, X=None, Y=None, scale=0.0)
    pts = eot.eot_cost(kind=2, d=3, n=8, m=8, ldc=0, C=None, X=p, Y=p, scale=2.0)
    info = eot.eot_grad_info(tol=1e-10, max_cg=100)

    def grad(cost, gC=None, ldg=8, gX=None, info_p=ctypes.byref(info), wS=1.0):
        return L.eot_gradient(ctypes.byref(cost), 0.1, p, p, 1.0, wS, gC, ldg, gX, None, None,
                              None, info_p, 0, p, 1 << 20, None)

    assert grad(dense, info_p=None) == eot.EOT_ERR_INVALID_ARG
    assert grad(pts, gC=p) == eot.EOT_ERR_INVALID_ARG            # no dense cotangent for points
    assert grad(dense, gX=p) == eot.EOT_ERR_INVALID_ARG          # no point gradient for dense
    assert grad(dense, gC=p, ldg=4) == eot.EOT_ERR_INVALID_ARG   # ldg < m
    info.tol = 0.0
    assert grad(dense) == eot.EOT_ERR_INVALID_ARG                # S needs a CG tolerance
    # point clouds: d in {2, 3}, positive finite scale, non-null points
    sz = ctypes.c_size_t(0)
    for d, scale, st in ((3, 2.0, eot.EOT_OK), (2, 1.0, eot.EOT_OK), (4, 1.0, eot.EOT_ERR_UNSUPPORTED),
                         (3, 0.0, eot.EOT_ERR_INVALID_ARG), (3, float("inf"), eot.EOT_ERR_INVALID_ARG)):
        pts.d, pts.scale = d, scale
        assert L.eot_workspace_size(eot.EOT_OP_GRADIENT, ctypes.byref(pts), 0, ctypes.byref(sz)) == st
    pts.d, pts.scale, pts.X = 3, 1.0, None
    assert L.eot_workspace_size(0, ctypes.byref(pts), 0, ctypes.byref(sz)) == eot.EOT_ERR_INVALID_ARG


def test_binding_rejects_cpu_tensors():
    import torch
    from paper_2504_02067_amd import eot
    with pytest.raises(ValueError):
        eot.make_cost(torch.zeros(4, 4))


def test_rows_per_tile_override_validation(L):
    from paper_2504_02067_amd import eot
    for bad in (7, 12, 512, -8):
        assert L.eot_set_rows_per_tile(bad) == eot.EOT_ERR_INVALID_ARG
    sz = ctypes.c_size_t(0)
    c = eot.eot_cost(kind=0, d=0, n=4096, m=4096, ldc=4096, C=ctypes.c_void_p(4096), X=None,
                     Y=None, scale=0.0)
    sizes = []
    for rb in (8, 256, 0):
        assert L.eot_set_rows_per_tile(rb) == eot.EOT_OK
        assert L.eot_workspace_size(eot.EOT_OP_SOLVE, ctypes.byref(c), 0, ctypes.byref(sz)) == 0
        sizes.append(sz.value)
    assert sizes[0] > sizes[1]          # 8-row tiles need more column partials


def test_batched_validation(L):
    """eot_solve_batched / eot_workspace_size_batched reject bad arguments before
    touching any device memory (the pointers below are never dereferenced)."""
    from paper_2504_02067_amd import eot
    p = ctypes.c_void_p(4096)
    cost = eot.eot_cost(kind=0, d=0, n=16, m=24, ldc=24, C=p, X=None, Y=None, scale=0.0)
    probs = (eot.eot_batch_problem * 2)()
    for k in range(2):
        probs[k] = eot.eot_batch_problem(cost=cost, r=p, c=p, f=p, g=p)
    o = eot.eot_solve_opts()
    L.eot_solve_opts_default(ctypes.byref(o))
    stats = (eot.eot_solve_stats * 2)()
    status = (ctypes.c_int32 * 2)()
    sz = ctypes.c_size_t(0)
    assert L.eot_workspace_size_batched(2, probs, 4, ctypes.byref(sz)) == eot.EOT_OK
    assert sz.value > 0
    # more workers never need less workspace
    sz1 = ctypes.c_size_t(0)
    assert L.eot_workspace_size_batched(2, probs, 1, ctypes.byref(sz1)) == eot.EOT_OK
    assert sz.value >= sz1.value

    def solve(nprob=2, pr=probs, workers=4, ws=p, nbytes=1 << 40):
        return L.eot_solve_batched(nprob, pr, ctypes.byref(o), workers, stats, status, ws,
                                   nbytes, None)

    assert solve(nprob=0) == eot.EOT_ERR_INVALID_ARG
    assert solve(workers=0) == eot.EOT_ERR_INVALID_ARG
    assert solve(pr=None) == eot.EOT_ERR_INVALID_ARG
    assert solve(ws=None) == eot.EOT_ERR_WORKSPACE
    assert solve(nbytes=16) == eot.EOT_ERR_WORKSPACE
    probs[1].r = None
    assert solve() == eot.EOT_ERR_INVALID_ARG
    probs[1].r = p
    probs[1].cost.n = 0
    assert solve() == eot.EOT_ERR_INVALID_ARG
    assert L.eot_workspace_size_batched(2, probs, 4, ctypes.byref(sz)) == eot.EOT_ERR_INVALID_ARG


def test_gradient_batched_validation(L):
    """eot_gradient_batched checks every problem's arguments (those of
    eot_gradient) and the workspace before any device work."""
    from paper_2504_02067_amd import eot
    p = ctypes.c_void_p(4096)
    c = eot.eot_cost(kind=0, d=0, n=8, m=8, ldc=8, C=p, X=None, Y=None, scale=0.0)
    probs = (eot.eot_grad_problem * 2)()
    for k in range(2):
        probs[k].cost = c
        probs[k].gamma = 0.1
        probs[k].f = p
        probs[k].g = p
        probs[k].ldg = 8
    info = (eot.eot_grad_info * 2)()
    for k in range(2):
        info[k].tol = 1e-10
        info[k].max_cg = 100
    nbytes = ctypes.c_size_t(0)
    assert L.eot_workspace_size_gradient_batched(2, probs, 4, ctypes.byref(nbytes)) == eot.EOT_OK
    one = ctypes.c_size_t(0)
    assert L.eot_workspace_size(eot.EOT_OP_GRADIENT, ctypes.byref(c), 0, ctypes.byref(one)) == 0
    assert nbytes.value >= 2 * one.value
    gb = L.eot_gradient_batched
    assert gb(0, probs, 1.0, 1.0, info, 0, 4, None, p, 1 << 30, None) == eot.EOT_ERR_INVALID_ARG
    assert gb(2, probs, 1.0, 1.0, None, 0, 4, None, p, 1 << 30, None) == eot.EOT_ERR_INVALID_ARG
    assert gb(2, probs, 1.0, 1.0, info, 0, 0, None, p, 1 << 30, None) == eot.EOT_ERR_INVALID_ARG
    assert gb(2, probs, float("nan"), 1.0, info, 0, 4, None, p, 1 << 30,
              None) == eot.EOT_ERR_INVALID_ARG
    probs[1].gamma = 0.0                      # one bad problem fails the call up front
    assert gb(2, probs, 1.0, 1.0, info, 0, 4, None, p, 1 << 30, None) == eot.EOT_ERR_INVALID_ARG
    probs[1].gamma = 0.1
    probs[1].grad_X = p                       # point gradients of a dense cost
    assert gb(2, probs, 1.0, 1.0, info, 0, 4, None, p, 1 << 30, None) == eot.EOT_ERR_INVALID_ARG
    probs[1].grad_X = None
    info[1].max_cg = 0                        # the S part needs a CG budget
    assert gb(2, probs, 1.0, 1.0, info, 0, 4, None, p, 1 << 30, None) == eot.EOT_ERR_INVALID_ARG
    info[1].max_cg = 100
    assert gb(2, probs, 1.0, 1.0, info, 0, 4, None, p, 16, None) == eot.EOT_ERR_WORKSPACE
    assert gb(2, probs, 1.0, 1.0, info, 0, 4, None, ctypes.c_void_p(4100), 1 << 30,
              None) == eot.EOT_ERR_WORKSPACE


def test_noalloc_hvp_rejects_oversize_before_device_work(L):
    """eot_hvp_noalloc checks the scratch it needs against its fixed 64 MiB
    before any HIP call: a dense 32768^2 cost needs 98 MiB."""
    from paper_2504_02067_amd import eot
    big = eot.eot_cost(kind=0, d=0, n=32768, m=32768, ldc=32768, C=ctypes.c_void_p(4096),
                       X=None, Y=None, scale=0.0)
    p = ctypes.c_void_p(8)
    assert L.eot_hvp_noalloc(ctypes.byref(big), 0.1, p, p, None, 0.5, p, p, p, p, 1,
                             None) == eot.EOT_ERR_WORKSPACE
    assert L.eot_hvp_noalloc(ctypes.byref(big), 0.1, None, p, None, 0.5, p, p, p, p, 1,
                             None) == eot.EOT_ERR_INVALID_ARG
