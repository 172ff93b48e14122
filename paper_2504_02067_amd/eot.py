"""Thin ctypes binding of libeot.so (include/eot.h) with the same names.

Arguments are torch tensors on the GPU; this module only checks shapes and
dtypes, allocates the workspace with torch, and forwards raw device
pointers and the current HIP stream. Every computation happens in the HIP
library; if it is not built, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libeot.so")

EOT_OK = 0
EOT_ERR_INVALID_ARG = 1
EOT_ERR_BAD_MARGINALS = 2
EOT_ERR_NONFINITE = 3
EOT_ERR_NOT_CONVERGED = 4
EOT_ERR_WORKSPACE = 5
EOT_ERR_UNSUPPORTED = 6
EOT_ERR_HIP = 7

EOT_PREC_FP64 = 0
EOT_PREC_MIXED = 1
EOT_COST_DENSE_F32 = 0
EOT_COST_DENSE_F64 = 1
EOT_COST_SQEUCLID_POINTS = 2
EOT_OP_MARGINALS = 0
EOT_OP_HVP = 1
EOT_OP_NEWTON_CG = 2
EOT_OP_SOLVE = 3
EOT_OP_GRADIENT = 4
EOT_OP_ROUND = 5
EOT_PROJ_TNP = 0
EOT_PROJ_SINKHORN = 1

_c_i32, _c_i64, _c_f64, _c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class eot_cost(ctypes.Structure):
    _fields_ = [("kind", _c_i32), ("d", _c_i32), ("n", _c_i64), ("m", _c_i64), ("ldc", _c_i64),
                ("C", _c_vp), ("X", _c_vp), ("Y", _c_vp), ("scale", _c_f64)]


class eot_newton_stats(ctypes.Structure):
    _fields_ = [("rho_out", _c_f64), ("cg_iters", _c_i32), ("levels", _c_i32),
                ("forcing_miss", _c_i32), ("status", _c_i32), ("passes", _c_i64),
                ("forcing_ratio", _c_f64)]


class eot_solve_opts(ctypes.Structure):
    _fields_ = [("gamma_init", _c_f64), ("gamma_final", _c_f64), ("tol", _c_f64), ("p", _c_f64),
                ("q1", _c_f64), ("w_r", _c_f64), ("adaptive_q", _c_i32),
                ("adaptive_rho0", _c_i32), ("max_cg", _c_i32), ("max_levels", _c_i32),
                ("max_backtrack", _c_i32), ("max_newton", _c_i32), ("max_sinkhorn", _c_i32),
                ("max_mdot", _c_i32), ("precision", _c_i32), ("verify_fp64", _c_i32),
                ("projection", _c_i32), ("cg_graph", _c_i32), ("verbose", _c_i32),
                ("warm_start", _c_i32), ("batch_persistent", _c_i32)]


class eot_solve_stats(ctypes.Structure):
    _fields_ = [("status", _c_i32), ("mdot_steps", _c_i32), ("newton_steps", _c_i32),
                ("cg_iters", _c_i32), ("backtracks", _c_i32), ("sinkhorn_iters", _c_i32),
                ("levels", _c_i32), ("forcing_misses", _c_i32), ("range_retries", _c_i32),
                ("mixed_stalls", _c_i32), ("linesearch_unresolved", _c_i32),
                ("passes_newton", _c_i64), ("passes_linesearch", _c_i64),
                ("passes_sinkhorn", _c_i64), ("passes_projection", _c_i64),
                ("passes_other", _c_i64), ("final_gamma", _c_f64), ("err_r", _c_f64),
                ("err_c", _c_f64), ("cost", _c_f64), ("dual_value", _c_f64),
                ("rho_last", _c_f64), ("delta_min_last", _c_f64), ("seconds", _c_f64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class eot_solve_state(ctypes.Structure):
    _fields_ = [("t", _c_i32), ("beta", _c_f64), ("beta_prev", _c_f64), ("q", _c_f64),
                ("rho0", _c_f64), ("u", _c_vp), ("v", _c_vp), ("u_prev", _c_vp),
                ("v_prev", _c_vp)]


_c_dp = ctypes.POINTER(ctypes.c_double)
_c_ip = ctypes.POINTER(ctypes.c_int32)
TRACE_STEP_FIELDS = ("beta", "eps_d", "start_err", "delta_min", "q", "newton", "sweeps")
TRACE_NEWTON_FIELDS = ("step_of", "gnorm", "eta", "cg_tol", "rho0", "rho_out", "cg_iters",
                       "levels", "alpha", "gnorm_next")
TRACE_INT_FIELDS = ("newton", "sweeps", "step_of", "cg_iters", "levels")


class eot_solve_trace(ctypes.Structure):
    _fields_ = ([("cap_steps", _c_i32), ("cap_newton", _c_i32), ("n_steps", _c_i32),
                 ("n_newton", _c_i32)]
                + [(k, _c_ip if k in TRACE_INT_FIELDS else _c_dp) for k in TRACE_STEP_FIELDS]
                + [(k, _c_ip if k in TRACE_INT_FIELDS else _c_dp) for k in TRACE_NEWTON_FIELDS])


# Every entry point declared in include/eot.h, with its ctypes signature.
class eot_batch_problem(ctypes.Structure):
    _fields_ = [("cost", eot_cost), ("r", _c_vp), ("c", _c_vp), ("f", _c_vp), ("g", _c_vp)]


class eot_round_info(ctypes.Structure):
    _fields_ = [("cost_round", _c_f64), ("cost_plan", _c_f64), ("err_r", _c_f64),
                ("err_c", _c_f64), ("mass_fix", _c_f64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class eot_grad_info(ctypes.Structure):
    _fields_ = [("tol", _c_f64), ("max_cg", _c_i32), ("cg_iters", _c_i32),
                ("cg_residual", _c_f64), ("S", _c_f64)]


class eot_grad_problem(ctypes.Structure):
    _fields_ = [("cost", eot_cost), ("gamma", _c_f64), ("f", _c_vp), ("g", _c_vp),
                ("grad_C", _c_vp), ("ldg", _c_i64), ("grad_X", _c_vp), ("grad_Y", _c_vp),
                ("grad_r", _c_vp), ("grad_c", _c_vp)]


SIGNATURES = {
    "eot_workspace_size": (_c_i32, [_c_i32, ctypes.POINTER(eot_cost), _c_i32,
                                    ctypes.POINTER(ctypes.c_size_t)]),
    "eot_marginals": (_c_i32, [ctypes.POINTER(eot_cost), _c_f64, _c_vp, _c_vp, _c_vp, _c_vp,
                               _c_vp, _c_vp, _c_vp, _c_vp, _c_i32, _c_vp, ctypes.c_size_t,
                               _c_vp]),
    "eot_hvp": (_c_i32, [ctypes.POINTER(eot_cost), _c_f64, _c_vp, _c_vp, _c_vp, _c_f64, _c_vp,
                         _c_vp, _c_vp, _c_vp, _c_i32, _c_vp, ctypes.c_size_t, _c_vp]),
    "eot_hvp_noalloc": (_c_i32, [ctypes.POINTER(eot_cost), _c_f64, _c_vp, _c_vp, _c_vp, _c_f64,
                                 _c_vp, _c_vp, _c_vp, _c_vp, _c_i32, _c_vp]),
    "eot_hvp_with_marginals": (_c_i32, [ctypes.POINTER(eot_cost), _c_f64, _c_vp, _c_vp, _c_vp,
                                        _c_vp, _c_f64, _c_vp, _c_vp, _c_vp, _c_vp, _c_i32, _c_vp,
                                        ctypes.c_size_t, _c_vp]),
    "eot_newton_cg": (_c_i32, [ctypes.POINTER(eot_cost), _c_f64, _c_vp, _c_vp, _c_vp, _c_vp,
                               _c_f64, _c_f64, _c_i32, _c_i32, _c_vp, _c_vp,
                               ctypes.POINTER(eot_newton_stats), _c_i32, _c_vp,
                               ctypes.c_size_t, _c_vp]),
    "eot_solve_opts_default": (None, [ctypes.POINTER(eot_solve_opts)]),
    "eot_solve": (_c_i32, [ctypes.POINTER(eot_cost), _c_vp, _c_vp,
                           ctypes.POINTER(eot_solve_opts), _c_vp, _c_vp,
                           ctypes.POINTER(eot_solve_stats), _c_vp, ctypes.c_size_t, _c_vp]),
    "eot_solve_ex": (_c_i32, [ctypes.POINTER(eot_cost), _c_vp, _c_vp,
                              ctypes.POINTER(eot_solve_opts), ctypes.POINTER(eot_solve_state),
                              ctypes.POINTER(eot_solve_state), ctypes.POINTER(eot_solve_trace),
                              _c_vp, _c_vp, ctypes.POINTER(eot_solve_stats), _c_vp,
                              ctypes.c_size_t, _c_vp]),
    "eot_workspace_size_batched": (_c_i32, [_c_i32, ctypes.POINTER(eot_batch_problem), _c_i32,
                                            ctypes.POINTER(ctypes.c_size_t)]),
    "eot_solve_batched": (_c_i32, [_c_i32, ctypes.POINTER(eot_batch_problem),
                                   ctypes.POINTER(eot_solve_opts), _c_i32,
                                   ctypes.POINTER(eot_solve_stats), ctypes.POINTER(_c_i32), _c_vp,
                                   ctypes.c_size_t, _c_vp]),
    "eot_round": (_c_i32, [ctypes.POINTER(eot_cost), _c_f64, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                           _c_vp, _c_vp, _c_vp, _c_vp, _c_i64, ctypes.POINTER(eot_round_info),
                           _c_vp, ctypes.c_size_t, _c_vp]),
    "eot_gradient": (_c_i32, [ctypes.POINTER(eot_cost), _c_f64, _c_vp, _c_vp, _c_f64, _c_f64,
                              _c_vp, _c_i64, _c_vp, _c_vp, _c_vp, _c_vp,
                              ctypes.POINTER(eot_grad_info), _c_i32, _c_vp, ctypes.c_size_t,
                              _c_vp]),
    "eot_workspace_size_gradient_batched": (_c_i32, [_c_i32, ctypes.POINTER(eot_grad_problem),
                                                     _c_i32, ctypes.POINTER(ctypes.c_size_t)]),
    "eot_gradient_batched": (_c_i32, [_c_i32, ctypes.POINTER(eot_grad_problem), _c_f64, _c_f64,
                                      ctypes.POINTER(eot_grad_info), _c_i32, _c_i32,
                                      ctypes.POINTER(_c_i32), _c_vp, ctypes.c_size_t, _c_vp]),
    "eot_set_rows_per_tile": (_c_i32, [_c_i32]),
    "eot_set_team_size": (_c_i32, [_c_i32, _c_i64]),
    "eot_set_cg_persist": (_c_i32, [_c_i32, _c_i32]),
    "eot_pass_timing": (_c_i32, [_c_i32]),
    "eot_pass_timing_read": (_c_i32, [_c_i32, _c_i32, _c_i32, _c_i32, ctypes.POINTER(_c_i64),
                                      ctypes.POINTER(_c_f64)]),
    "eot_status_string": (ctypes.c_char_p, [_c_i32]),
    "eot_version": (ctypes.c_char_p, []),
}

_lib = None


class EotError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


def lib() -> ctypes.CDLL:
    """Load libeot.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2504_02067_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().eot_status_string(int(status)).decode()


def version() -> str:
    return lib().eot_version().decode()


def _check(status: int, where: str, allow=(EOT_OK,)):
    if status not in allow:
        raise EotError(status, where)
    return status


def _vec(t: Optional[torch.Tensor], k: int, name: str, optional: bool = False):
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == k):
        raise ValueError(f"{name}: need a contiguous float64 GPU tensor of {k} elements")
    return ctypes.c_void_p(t.data_ptr())


class PointCloud:
    """Squared-Euclidean cost between point clouds, recomputed inside every pass:
    C_ij = |X_i - Y_j|^2 / scale with X (n x d) and Y (m x d) float32 GPU
    tensors, d in {2, 3} (difference form on the vector units) or d in
    {16, 32, 48, 64} (x . y on the matrix cores in mixed precision). The n x m
    matrix is never stored."""

    def __init__(self, X: torch.Tensor, Y: torch.Tensor, scale: float):
        for name, T in (("X", X), ("Y", Y)):
            if not T.is_cuda or T.dim() != 2 or T.dtype != torch.float32 or not T.is_contiguous():
                raise ValueError(f"{name}: need a contiguous 2-D float32 GPU tensor")
        if X.shape[1] != Y.shape[1] or X.shape[1] not in (2, 3, 16, 32, 48, 64):
            raise ValueError("X and Y need the same dimension d in {2, 3, 16, 32, 48, 64}")
        if not scale > 0:
            raise ValueError("scale must be positive")
        self.X, self.Y, self.scale = X, Y, float(scale)
        self.device = X.device
        self.shape = (X.shape[0], Y.shape[0])


def make_cost(C) -> eot_cost:
    """Cost descriptor: a 2-D float32 / float64 GPU tensor (row stride >= columns,
    unit column stride) or a PointCloud."""
    if isinstance(C, PointCloud):
        return eot_cost(kind=EOT_COST_SQEUCLID_POINTS, d=C.X.shape[1], n=C.shape[0],
                        m=C.shape[1], ldc=0, C=None, X=ctypes.c_void_p(C.X.data_ptr()),
                        Y=ctypes.c_void_p(C.Y.data_ptr()), scale=C.scale)
    if not C.is_cuda or C.dim() != 2 or C.stride(1) != 1 or C.stride(0) < C.shape[1]:
        raise ValueError("C: need a 2-D GPU tensor with unit column stride")
    if C.dtype == torch.float32:
        kind = EOT_COST_DENSE_F32
    elif C.dtype == torch.float64:
        kind = EOT_COST_DENSE_F64
    else:
        raise ValueError("C must be float32 or float64")
    return eot_cost(kind=kind, d=0, n=C.shape[0], m=C.shape[1], ldc=C.stride(0),
                    C=ctypes.c_void_p(C.data_ptr()), X=None, Y=None, scale=0.0)


def _prec(precision) -> int:
    if precision in ("fp64", EOT_PREC_FP64):
        return EOT_PREC_FP64
    if precision in ("mixed", EOT_PREC_MIXED):
        return EOT_PREC_MIXED
    raise ValueError(precision)


def workspace(op: int, cost: eot_cost, prec: int, device) -> torch.Tensor:
    nbytes = ctypes.c_size_t(0)
    _check(lib().eot_workspace_size(op, ctypes.byref(cost), prec, ctypes.byref(nbytes)),
           "eot_workspace_size")
    buf = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + int(nbytes.value)]


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def eot_marginals(C, gamma, f, g, row_shift=None, c_for_s=None, precision="fp64",
                  want=("log_rP", "log_cP", "mass")):
    """log r(P), log c(P), sum P and (with c_for_s) s_i = sum_j P_ij^2 / c_j."""
    cost = make_cost(C)
    n, m = cost.n, cost.m
    dev = C.device
    prec = _prec(precision)
    out = {}
    lr = torch.empty(n, dtype=torch.float64, device=dev) if "log_rP" in want else None
    lc = torch.empty(m, dtype=torch.float64, device=dev) if "log_cP" in want else None
    ms = torch.empty(1, dtype=torch.float64, device=dev) if "mass" in want else None
    s = torch.empty(n, dtype=torch.float64, device=dev) if c_for_s is not None else None
    ws = workspace(EOT_OP_MARGINALS, cost, prec, dev)
    st = lib().eot_marginals(ctypes.byref(cost), float(gamma), _vec(f, n, "f"), _vec(g, m, "g"),
                             _vec(row_shift, n, "row_shift", True),
                             _vec(lr, n, "log_rP", True), _vec(lc, m, "log_cP", True),
                             _vec(ms, 1, "mass", True), _vec(c_for_s, m, "c_for_s", True),
                             _vec(s, n, "s", True), prec, ctypes.c_void_p(ws.data_ptr()),
                             ws.numel(), _stream(dev))
    _check(st, "eot_marginals")
    out.update(log_rP=lr, log_cP=lc, mass=ms, s=s)
    return out


def eot_hvp(C, gamma, f, g, rho, x, y, row_shift=None, precision="fp64"):
    """(Hx, Hy) = discounted Hessian of the dual times (x, y), log units."""
    cost = make_cost(C)
    n, m = cost.n, cost.m
    dev = C.device
    prec = _prec(precision)
    Hx = torch.empty(n, dtype=torch.float64, device=dev)
    Hy = torch.empty(m, dtype=torch.float64, device=dev)
    ws = workspace(EOT_OP_HVP, cost, prec, dev)
    st = lib().eot_hvp(ctypes.byref(cost), float(gamma), _vec(f, n, "f"), _vec(g, m, "g"),
                       _vec(row_shift, n, "row_shift", True), float(rho), _vec(x, n, "x"),
                       _vec(y, m, "y"), _vec(Hx, n, "Hx"), _vec(Hy, m, "Hy"), prec,
                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev))
    _check(st, "eot_hvp")
    return Hx, Hy


def eot_hvp_noalloc(C, gamma, f, g, rho, x, y, row_shift=None, precision="fp64", Hx=None, Hy=None):
    """eot_hvp on the library's own per-GPU scratch (no workspace argument; the
    call allocates nothing). Hx, Hy: optional preallocated outputs."""
    cost = make_cost(C)
    n, m = cost.n, cost.m
    dev = C.device
    prec = _prec(precision)
    Hx = torch.empty(n, dtype=torch.float64, device=dev) if Hx is None else Hx
    Hy = torch.empty(m, dtype=torch.float64, device=dev) if Hy is None else Hy
    st = lib().eot_hvp_noalloc(ctypes.byref(cost), float(gamma), _vec(f, n, "f"), _vec(g, m, "g"),
                               _vec(row_shift, n, "row_shift", True), float(rho), _vec(x, n, "x"),
                               _vec(y, m, "y"), _vec(Hx, n, "Hx"), _vec(Hy, m, "Hy"), prec,
                               _stream(dev))
    _check(st, "eot_hvp_noalloc")
    return Hx, Hy


def eot_hvp_with_marginals(C, gamma, f, g, log_rP, log_cP, rho, x, y, precision="fp64"):
    """(Hx, Hy) = discounted Hessian times (x, y) with the diagonal blocks
    exp(log_rP), exp(log_cP) given (log_rP is also the row shift)."""
    cost = make_cost(C)
    n, m = cost.n, cost.m
    dev = C.device
    prec = _prec(precision)
    Hx = torch.empty(n, dtype=torch.float64, device=dev)
    Hy = torch.empty(m, dtype=torch.float64, device=dev)
    ws = workspace(EOT_OP_HVP, cost, prec, dev)
    st = lib().eot_hvp_with_marginals(ctypes.byref(cost), float(gamma), _vec(f, n, "f"),
                                      _vec(g, m, "g"), _vec(log_rP, n, "log_rP"),
                                      _vec(log_cP, m, "log_cP"), float(rho), _vec(x, n, "x"),
                                      _vec(y, m, "y"), _vec(Hx, n, "Hx"), _vec(Hy, m, "Hy"), prec,
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev))
    _check(st, "eot_hvp_with_marginals")
    return Hx, Hy


@dataclass
class NewtonOut:
    dir_f: torch.Tensor
    dir_g: torch.Tensor
    rho_out: float
    cg_iters: int
    levels: int
    forcing_miss: int
    passes: int
    forcing_ratio: float


def eot_newton_cg(C, gamma, f, g, r, c, eta, rho0=0.0, max_cg=1000, max_levels=30,
                  precision="fp64"):
    """NewtonSolve (Alg. 2) at (f, g) with c(P) = c; direction in cost units."""
    cost = make_cost(C)
    n, m = cost.n, cost.m
    dev = C.device
    prec = _prec(precision)
    df = torch.empty(n, dtype=torch.float64, device=dev)
    dg = torch.empty(m, dtype=torch.float64, device=dev)
    stats = eot_newton_stats()
    ws = workspace(EOT_OP_NEWTON_CG, cost, prec, dev)
    st = lib().eot_newton_cg(ctypes.byref(cost), float(gamma), _vec(f, n, "f"), _vec(g, m, "g"),
                             _vec(r, n, "r"), _vec(c, m, "c"), float(eta), float(rho0),
                             int(max_cg), int(max_levels), _vec(df, n, "dir_f"),
                             _vec(dg, m, "dir_g"), ctypes.byref(stats), prec,
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev))
    _check(st, "eot_newton_cg")
    return NewtonOut(df, dg, stats.rho_out, stats.cg_iters, stats.levels, stats.forcing_miss,
                     stats.passes, stats.forcing_ratio)


def default_solve_opts(**kw) -> eot_solve_opts:
    o = eot_solve_opts()
    lib().eot_solve_opts_default(ctypes.byref(o))
    names = {k for k, _ in eot_solve_opts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown solve option {k!r}")
        if k == "precision":
            v = _prec(v)
        if k == "projection":
            v = {"tnp": EOT_PROJ_TNP, "sinkhorn": EOT_PROJ_SINKHORN}.get(v, v)
        setattr(o, k, v)
    return o


def eot_solve(C, r, c, opts: Optional[eot_solve_opts] = None, allow_not_converged=False, **kw):
    """MDOT + TruncatedNewtonProject; returns (f, g, stats dict)."""
    cost = make_cost(C)
    n, m = cost.n, cost.m
    dev = C.device
    o = opts if opts is not None else default_solve_opts(**kw)
    f = torch.empty(n, dtype=torch.float64, device=dev)
    g = torch.empty(m, dtype=torch.float64, device=dev)
    stats = eot_solve_stats()
    ws = workspace(EOT_OP_SOLVE, cost, o.precision, dev)
    st = lib().eot_solve(ctypes.byref(cost), _vec(r, n, "r"), _vec(c, m, "c"), ctypes.byref(o),
                         _vec(f, n, "f"), _vec(g, m, "g"), ctypes.byref(stats),
                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev))
    allow = (EOT_OK, EOT_ERR_NOT_CONVERGED) if allow_not_converged else (EOT_OK,)
    _check(st, "eot_solve", allow)
    return f, g, stats.as_dict()


def eot_solve_ex(C, r, c, opts: Optional[eot_solve_opts] = None, warm=None, resume=None,
                 want_state=False, trace=False, cap_steps=512, cap_newton=4096,
                 allow_not_converged=False, **kw):
    """eot_solve with the carried MDOT state and the step trace.

    warm: (f0, g0) cost-unit potentials that start the first projection
    (sets opts.warm_start); resume: a state dict returned by an earlier call
    (device vectors in log units). Returns (f, g, stats dict, trace dict or
    None, state dict or None)."""
    import numpy as np
    cost = make_cost(C)
    n, m = cost.n, cost.m
    dev = C.device
    o = opts if opts is not None else default_solve_opts(**kw)
    f = torch.empty(n, dtype=torch.float64, device=dev)
    g = torch.empty(m, dtype=torch.float64, device=dev)
    if warm is not None:
        f.copy_(warm[0])
        g.copy_(warm[1])
        o.warm_start = 1
    stats = eot_solve_stats()
    rs = None
    if resume is not None:
        rs = eot_solve_state(t=resume["t"], beta=resume["beta"], beta_prev=resume["beta_prev"],
                             q=resume["q"], rho0=resume["rho0"],
                             u=_vec(resume["u"], n, "u"), v=_vec(resume["v"], m, "v"),
                             u_prev=_vec(resume["u_prev"], n, "u_prev"),
                             v_prev=_vec(resume["v_prev"], m, "v_prev"))
    so, sv = None, None
    if want_state:
        sv = {k: torch.empty(n if k in ("u", "u_prev") else m, dtype=torch.float64, device=dev)
              for k in ("u", "v", "u_prev", "v_prev")}
        so = eot_solve_state(**{k: _vec(t, t.numel(), k) for k, t in sv.items()})
    tr, bufs = None, None
    if trace:
        tr = eot_solve_trace(cap_steps=cap_steps, cap_newton=cap_newton)
        bufs = {}
        for k in TRACE_STEP_FIELDS + TRACE_NEWTON_FIELDS:
            cap = cap_steps if k in TRACE_STEP_FIELDS else cap_newton
            a = np.zeros(cap, dtype=np.int32 if k in TRACE_INT_FIELDS else np.float64)
            bufs[k] = a
            setattr(tr, k, a.ctypes.data_as(_c_ip if k in TRACE_INT_FIELDS else _c_dp))
    ws = workspace(EOT_OP_SOLVE, cost, o.precision, dev)
    st = lib().eot_solve_ex(ctypes.byref(cost), _vec(r, n, "r"), _vec(c, m, "c"),
                            ctypes.byref(o), ctypes.byref(rs) if rs is not None else None,
                            ctypes.byref(so) if so is not None else None,
                            ctypes.byref(tr) if tr is not None else None,
                            _vec(f, n, "f"), _vec(g, m, "g"), ctypes.byref(stats),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev))
    allow = (EOT_OK, EOT_ERR_NOT_CONVERGED) if allow_not_converged else (EOT_OK,)
    _check(st, "eot_solve_ex", allow)
    d = stats.as_dict()
    d["status"] = int(st)
    tdict = None
    if tr is not None:
        ns, nk = min(tr.n_steps, cap_steps), min(tr.n_newton, cap_newton)
        tdict = {"n_steps": tr.n_steps, "n_newton": tr.n_newton}
        for k in TRACE_STEP_FIELDS:
            tdict[k] = bufs[k][:ns].copy()
        for k in TRACE_NEWTON_FIELDS:
            tdict[k] = bufs[k][:nk].copy()
    sdict = None
    if so is not None:
        sdict = {"t": so.t, "beta": so.beta, "beta_prev": so.beta_prev, "q": so.q,
                 "rho0": so.rho0, **sv}
    return f, g, d, tdict, sdict


def eot_solve_batched(problems, opts: Optional[eot_solve_opts] = None, workers=8,
                      allow_not_converged=False, check=True, **kw):
    """Solve many problems at once. ``problems``: sequence of (C, r, c) with C a
    dense GPU tensor or a PointCloud. Returns (list of (f, g), list of stats
    dicts, list of status codes); with check=False a failed problem does not
    raise (its status says what happened)."""
    k = len(problems)
    o = opts if opts is not None else default_solve_opts(**kw)
    arr = (eot_batch_problem * k)()
    outs, keep = [], []
    dev = None
    for i, (C, r, c) in enumerate(problems):
        cost = make_cost(C)
        dev = C.device
        f = torch.empty(cost.n, dtype=torch.float64, device=dev)
        g = torch.empty(cost.m, dtype=torch.float64, device=dev)
        arr[i].cost = cost
        arr[i].r = _vec(r, cost.n, "r")
        arr[i].c = _vec(c, cost.m, "c")
        arr[i].f = _vec(f, cost.n, "f")
        arr[i].g = _vec(g, cost.m, "g")
        outs.append((f, g))
        keep.append((C, r, c))
    nbytes = ctypes.c_size_t(0)
    _check(lib().eot_workspace_size_batched(k, arr, int(workers), ctypes.byref(nbytes)),
           "eot_workspace_size_batched")
    buf = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
    off = (-buf.data_ptr()) % 256
    ws = buf[off:off + int(nbytes.value)]
    stats = (eot_solve_stats * k)()
    status = (_c_i32 * k)()
    st = lib().eot_solve_batched(k, arr, ctypes.byref(o), int(workers), stats, status,
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev))
    allow = (EOT_OK, EOT_ERR_NOT_CONVERGED) if allow_not_converged else (EOT_OK,)
    if check:
        _check(st, "eot_solve_batched", allow)
    return outs, [stats[i].as_dict() for i in range(k)], [int(status[i]) for i in range(k)]


def eot_round(C, gamma, f, g, r, c, plan=False):
    """Rounding of the plan at (f, g) onto U(r, c). Returns a dict with x, y, er,
    ec (the implicit rounded plan D(x) P D(y) + er ec^T / |er|_1), the dense
    rounded plan when ``plan`` (dense costs only) and the eot_round_info
    fields."""
    cost = make_cost(C)
    n, m = cost.n, cost.m
    dev = C.device
    out = {k: torch.empty(sz, dtype=torch.float64, device=dev)
           for k, sz in (("x", n), ("y", m), ("er", n), ("ec", m))}
    out["plan"] = torch.empty((n, m), dtype=torch.float64, device=dev) if plan else None
    info = eot_round_info()
    ws = workspace(EOT_OP_ROUND, cost, EOT_PREC_FP64, dev)
    P = out["plan"]
    st = lib().eot_round(ctypes.byref(cost), float(gamma), _vec(f, n, "f"), _vec(g, m, "g"),
                         _vec(r, n, "r"), _vec(c, m, "c"), _vec(out["x"], n, "x"),
                         _vec(out["y"], m, "y"), _vec(out["er"], n, "er"), _vec(out["ec"], m, "ec"),
                         None if P is None else ctypes.c_void_p(P.data_ptr()), m,
                         ctypes.byref(info), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                         _stream(dev))
    _check(st, "eot_round")
    out.update(info.as_dict())
    return out


def eot_gradient(C, gamma, f, g, w_W=1.0, w_S=0.0, want=None, tol=1e-11, max_cg=5000,
                 precision="fp64", allow_not_converged=False):
    """Vector-Jacobian product of (W, S) at potentials (f, g) with weights
    (w_W, w_S). ``want`` names the outputs among "C" (dense costs), "X", "Y"
    (point clouds), "r", "c"; returns a dict of FP64 tensors plus "S",
    "cg_iters" and "cg_residual"."""
    cost = make_cost(C)
    n, m = cost.n, cost.m
    dev = C.device
    pts = cost.kind == EOT_COST_SQEUCLID_POINTS
    if want is None:
        want = ("X", "Y", "r", "c") if pts else ("C", "r", "c")
    d = cost.d
    out = {}
    out["C"] = torch.empty((n, m), dtype=torch.float64, device=dev) if "C" in want else None
    out["X"] = torch.empty((n, d), dtype=torch.float64, device=dev) if "X" in want else None
    out["Y"] = torch.empty((m, d), dtype=torch.float64, device=dev) if "Y" in want else None
    out["r"] = torch.empty(n, dtype=torch.float64, device=dev) if "r" in want else None
    out["c"] = torch.empty(m, dtype=torch.float64, device=dev) if "c" in want else None
    info = eot_grad_info(tol=float(tol), max_cg=int(max_cg))
    prec = _prec(precision)
    ws = workspace(EOT_OP_GRADIENT, cost, prec, dev)

    def ptr(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    st = lib().eot_gradient(ctypes.byref(cost), float(gamma), _vec(f, n, "f"), _vec(g, m, "g"),
                            float(w_W), float(w_S), ptr(out["C"]), m, ptr(out["X"]),
                            ptr(out["Y"]), ptr(out["r"]), ptr(out["c"]), ctypes.byref(info),
                            prec, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(dev))
    allow = (EOT_OK, EOT_ERR_NOT_CONVERGED) if allow_not_converged else (EOT_OK,)
    _check(st, "eot_gradient", allow)
    out.update(S=info.S, cg_iters=info.cg_iters, cg_residual=info.cg_residual, status=st)
    return out


def eot_gradient_batched(problems, w_W=1.0, w_S=0.0, want=None, tol=1e-11, max_cg=5000,
                         precision="fp64", workers=8, check=True):
    """eot_gradient over many problems at once. ``problems``: sequence of
    (C, gamma, f, g) with C a dense GPU tensor or a PointCloud. Returns a list of
    per-problem dicts as eot_gradient's (tensors named by ``want``, plus "S",
    "cg_iters", "cg_residual" and "status"); with check=False a failed problem
    does not raise."""
    k = len(problems)
    arr = (eot_grad_problem * k)()
    info = (eot_grad_info * k)()
    outs, keep = [], []
    dev = None

    def ptr(t):
        return None if t is None else ctypes.c_void_p(t.data_ptr())

    for i, (C, gamma, f, g) in enumerate(problems):
        cost = make_cost(C)
        n, m, d = cost.n, cost.m, cost.d
        dev = C.device
        pts = cost.kind == EOT_COST_SQEUCLID_POINTS
        w = want if want is not None else (("X", "Y", "r", "c") if pts else ("C", "r", "c"))
        o = {"C": torch.empty((n, m), dtype=torch.float64, device=dev) if "C" in w else None,
             "X": torch.empty((n, d), dtype=torch.float64, device=dev) if "X" in w else None,
             "Y": torch.empty((m, d), dtype=torch.float64, device=dev) if "Y" in w else None,
             "r": torch.empty(n, dtype=torch.float64, device=dev) if "r" in w else None,
             "c": torch.empty(m, dtype=torch.float64, device=dev) if "c" in w else None}
        arr[i].cost = cost
        arr[i].gamma = float(gamma)
        arr[i].f = _vec(f, n, "f")
        arr[i].g = _vec(g, m, "g")
        arr[i].grad_C = ptr(o["C"])
        arr[i].ldg = m
        arr[i].grad_X = ptr(o["X"])
        arr[i].grad_Y = ptr(o["Y"])
        arr[i].grad_r = ptr(o["r"])
        arr[i].grad_c = ptr(o["c"])
        info[i].tol = float(tol)
        info[i].max_cg = int(max_cg)
        outs.append(o)
        keep.append((C, f, g))
    nbytes = ctypes.c_size_t(0)
    _check(lib().eot_workspace_size_gradient_batched(k, arr, int(workers), ctypes.byref(nbytes)),
           "eot_workspace_size_gradient_batched")
    buf = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
    off = (-buf.data_ptr()) % 256
    ws = buf[off:off + int(nbytes.value)]
    status = (_c_i32 * k)()
    st = lib().eot_gradient_batched(k, arr, float(w_W), float(w_S), info, _prec(precision),
                                    int(workers), status, ctypes.c_void_p(ws.data_ptr()),
                                    ws.numel(), _stream(dev))
    if check:
        _check(st, "eot_gradient_batched")
    for i, o in enumerate(outs):
        o.update(S=info[i].S, cg_iters=info[i].cg_iters, cg_residual=info[i].cg_residual,
                 status=int(status[i]))
    return outs


def eot_set_rows_per_tile(rows: int) -> None:
    """Force the tile height of the passes (power of two in [8, 256]); 0 restores
    the library's choice."""
    _check(lib().eot_set_rows_per_tile(int(rows)), "eot_set_rows_per_tile")


def eot_set_cg_persist(enable: int, grid: int = 0) -> None:
    """Single-launch CG of small problems on (1, default) or off (0); grid
    0 = default workgroup count."""
    _check(lib().eot_set_cg_persist(int(enable), int(grid)), "eot_set_cg_persist")


def eot_set_team_size(k: int, entries_per_wg: int = 0) -> None:
    _check(lib().eot_set_team_size(int(k), int(entries_per_wg)), "eot_set_team_size")


def eot_pass_timing(enable: bool) -> None:
    """Enable (and clear) or disable the library's per-pass event timer."""
    _check(lib().eot_pass_timing(1 if enable else 0), "eot_pass_timing")


def eot_pass_timing_read(nr=-1, nc=-1, precision=-1, fused_hvp=-1):
    """(launches, total milliseconds) of the recorded pass kernels matching the filter."""
    k = _c_i64(0)
    ms = _c_f64(0.0)
    prec = -1 if precision == -1 else _prec(precision)
    _check(lib().eot_pass_timing_read(int(nr), int(nc), prec, int(fused_hvp), ctypes.byref(k),
                                      ctypes.byref(ms)), "eot_pass_timing_read")
    return int(k.value), float(ms.value)
