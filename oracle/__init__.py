"""NumPy bindings of the FP64 CPU oracle (oracle/eot_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
CPU-baseline leg of bench.py; the product package never imports it.

Functions take the paper's log-unit potentials (u, v) and inverse
temperature beta, plus a dense cost C (any float dtype, promoted exactly to
float64). Helpers ``to_log_units`` / ``to_cost_units`` convert from/to the
library's cost-unit potentials f = u / beta, g = v / beta (temperature
gamma = 1 / beta), using the same single IEEE division u = f / gamma.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64
_f64 = ctypes.c_double
_i32 = ctypes.c_int32


class Opts(ctypes.Structure):
    _fields_ = [("gamma_init", _f64), ("gamma_final", _f64), ("tol", _f64),
                ("p", _f64), ("q1", _f64), ("w_r", _f64),
                ("adaptive_q", _i32), ("adaptive_rho0", _i32),
                ("max_cg", _i32), ("max_levels", _i32), ("max_backtrack", _i32),
                ("max_newton", _i32), ("max_sinkhorn", _i32), ("max_mdot", _i32),
                ("projection", _i32)]


class Stats(ctypes.Structure):
    _fields_ = [("status", _i32), ("mdot_steps", _i32), ("newton_steps", _i32),
                ("cg_iters", _i32), ("backtracks", _i32), ("sinkhorn_iters", _i32),
                ("levels", _i32), ("forcing_misses", _i32), ("linesearch_unresolved", _i32),
                ("passes_newton", ctypes.c_int64), ("passes_linesearch", ctypes.c_int64),
                ("passes_sinkhorn", ctypes.c_int64), ("passes_projection", ctypes.c_int64),
                ("final_beta", _f64), ("err_r", _f64), ("err_c", _f64),
                ("cost", _f64), ("dual_value", _f64), ("rho_last", _f64),
                ("delta_min_last", _f64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Trace(ctypes.Structure):
    _fields_ = [("cap_steps", _i32), ("cap_newton", _i32), ("n_steps", _i32),
                ("n_newton", _i32),
                ("beta", _dp), ("eps_d", _dp), ("start_err", _dp), ("delta_min", _dp),
                ("q", _dp), ("newton", _i32p), ("sweeps", _i32p), ("u_proj", _dp),
                ("v_proj", _dp),
                ("step_of", _i32p), ("gnorm", _dp), ("eta", _dp), ("cg_tol", _dp),
                ("rho0", _dp), ("rho_out", _dp), ("cg_iters", _i32p), ("levels", _i32p),
                ("alpha", _dp), ("gnorm_next", _dp)]


STEP_FIELDS = ("beta", "eps_d", "start_err", "delta_min", "q", "newton", "sweeps")
NEWTON_FIELDS = ("step_of", "gnorm", "eta", "cg_tol", "rho0", "rho_out", "cg_iters",
                 "levels", "alpha", "gnorm_next")
INT_FIELDS = ("newton", "sweeps", "step_of", "cg_iters", "levels")


class State(ctypes.Structure):
    _fields_ = [("t", _i32), ("beta", _f64), ("beta_prev", _f64), ("q", _f64),
                ("rho0", _f64), ("u", _dp), ("v", _dp), ("u_prev", _dp), ("v_prev", _dp)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        sig = {
            "orc_log_row_marginal": (None, [_i64, _i64, _dp, _f64, _dp, _dp, _dp]),
            "orc_log_col_marginal": (None, [_i64, _i64, _dp, _f64, _dp, _dp, _dp]),
            "orc_mass": (_f64, [_i64, _i64, _dp, _f64, _dp, _dp]),
            "orc_row_square_sum": (None, [_i64, _i64, _dp, _f64, _dp, _dp, _dp, _dp]),
            "orc_dual": (_f64, [_i64, _i64, _dp, _f64, _dp, _dp, _dp, _dp]),
            "orc_transport_cost": (_f64, [_i64, _i64, _dp, _f64, _dp, _dp]),
            "orc_hvp": (None, [_i64, _i64, _dp, _f64, _dp, _dp, _f64, _dp, _dp, _dp, _dp]),
            "orc_fr_apply": (None, [_i64, _i64, _dp, _f64, _dp, _dp, _dp, _dp, _f64, _dp, _dp]),
            "orc_pcg": (ctypes.c_int, [_i64, _i64, _dp, _f64, _dp, _dp, _dp, _dp, _dp,
                                       _f64, _dp, _f64, _i32, _dp, _i32p]),
            "orc_newton_solve": (ctypes.c_int, [_i64, _i64, _dp, _f64, _dp, _dp, _dp, _dp,
                                                _dp, _f64, _f64, _i32, _i32, _dp, _dp, _dp,
                                                _i32p, _i32p, _i64p, _i32p]),
            "orc_chi_sinkhorn": (ctypes.c_int, [_i64, _i64, _dp, _f64, _dp, _dp, _dp, _dp,
                                                _dp, _f64, _i32, _i32p]),
            "orc_line_search": (ctypes.c_int, [_i64, _i64, _dp, _f64, _dp, _dp, _dp, _dp,
                                               _dp, _i32, _dp, _dp, _i32p, _i32p]),
            "orc_tnp": (ctypes.c_int, [_i64, _i64, _dp, _f64, _dp, _dp, _dp, _dp, _f64,
                                       ctypes.POINTER(Opts), _dp, _dp, ctypes.POINTER(Stats)]),
            "orc_solve": (ctypes.c_int, [_i64, _i64, _dp, _dp, _dp, ctypes.POINTER(Opts),
                                         _dp, _dp, ctypes.POINTER(Stats)]),
            "orc_round": (None, [_i64, _i64, _dp, _f64, _dp, _dp, _dp, _dp, _dp]),
            "orc_solve_ex": (ctypes.c_int, [_i64, _i64, _dp, _dp, _dp, ctypes.POINTER(Opts),
                                            _i32, ctypes.POINTER(State),
                                            ctypes.POINTER(State), ctypes.POINTER(Trace),
                                            _dp, _dp, ctypes.POINTER(Stats)]),
            "orc_adjust_schedule": (_f64, [_f64, _f64]),
            "orc_extrapolate": (None, [_i64, _dp, _dp, _f64, _f64, _f64]),
            "orc_forcing_eta": (_f64, [_f64, _f64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _d(x):
    a = np.ascontiguousarray(x, dtype=np.float64)
    return a


def _p(a):
    return a.ctypes.data_as(_dp)


def _C(C):
    C = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    assert C.ndim == 2
    return C


# ---------------------------------------------------------------- units

def to_log_units(f, g, gamma):
    """u = f / gamma, v = g / gamma (one IEEE division each)."""
    f = _d(f); g = _d(g)
    return f / gamma, g / gamma


def to_cost_units(u, v, gamma):
    return _d(u) * gamma, _d(v) * gamma


def beta_of(gamma):
    return 1.0 / gamma


# ---------------------------------------------------------------- wrappers

def sqeuclid_points_cost(X, Y, scale, block=1024):
    """Dense FP64 cost of a point-cloud problem (Sec. 4.2, squared Euclidean
    ground cost): C_ij = sum_k (x_ik - y_jk)^2 / scale, evaluated in the
    difference form, row block by row block."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    C = np.empty((X.shape[0], Y.shape[0]))
    for i0 in range(0, X.shape[0], block):
        D = X[i0:i0 + block, None, :] - Y[None, :, :]
        C[i0:i0 + block] = (D * D).sum(-1) / scale
    return C


def log_row_marginal(C, beta, u, v):
    C = _C(C); u = _d(u); v = _d(v)
    out = np.empty(C.shape[0])
    lib().orc_log_row_marginal(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v), _p(out))
    return out


def log_col_marginal(C, beta, u, v):
    C = _C(C); u = _d(u); v = _d(v)
    out = np.empty(C.shape[1])
    lib().orc_log_col_marginal(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v), _p(out))
    return out


def mass(C, beta, u, v):
    C = _C(C); u = _d(u); v = _d(v)
    return lib().orc_mass(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v))


def row_square_sum(C, beta, u, v, c):
    C = _C(C); u = _d(u); v = _d(v); c = _d(c)
    out = np.empty(C.shape[0])
    lib().orc_row_square_sum(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v), _p(c), _p(out))
    return out


def dual(C, beta, u, v, r, c):
    C = _C(C); u = _d(u); v = _d(v); r = _d(r); c = _d(c)
    return lib().orc_dual(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v), _p(r), _p(c))


def transport_cost(C, beta, u, v):
    C = _C(C); u = _d(u); v = _d(v)
    return lib().orc_transport_cost(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v))


def hvp(C, beta, u, v, rho, x, y):
    C = _C(C); u = _d(u); v = _d(v); x = _d(x); y = _d(y)
    Hx = np.empty(C.shape[0]); Hy = np.empty(C.shape[1])
    lib().orc_hvp(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v), float(rho),
                  _p(x), _p(y), _p(Hx), _p(Hy))
    return Hx, Hy


def fr_apply(C, beta, u, v, rP, c, rho, p):
    C = _C(C); u = _d(u); v = _d(v); rP = _d(rP); c = _d(c); p = _d(p)
    out = np.empty(C.shape[0])
    lib().orc_fr_apply(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v), _p(rP), _p(c),
                       float(rho), _p(p), _p(out))
    return out


def pcg(C, beta, u, v, rP, c, s, rho, b, tol, max_iter=1000):
    C = _C(C); u = _d(u); v = _d(v); rP = _d(rP); c = _d(c); s = _d(s); b = _d(b)
    d = np.empty(C.shape[0])
    it = ctypes.c_int32(0)
    st = lib().orc_pcg(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v), _p(rP), _p(c),
                       _p(s), float(rho), _p(b), float(tol), int(max_iter), _p(d),
                       ctypes.byref(it))
    return d, int(it.value), int(st)


@dataclass
class NewtonResult:
    du: np.ndarray
    dv: np.ndarray
    rho: float
    cg_iters: int
    levels: int
    passes: int
    status: int
    forcing_miss: int


def newton_solve(C, beta, u, v, r, c, log_rP, eta, rho0=0.0, max_cg=1000, max_levels=30):
    C = _C(C); u = _d(u); v = _d(v); r = _d(r); c = _d(c); lr = _d(log_rP)
    n, m = C.shape
    du = np.empty(n); dv = np.empty(m)
    rho = ctypes.c_double(0.0)
    it = ctypes.c_int32(0); lev = ctypes.c_int32(0); np_ = ctypes.c_int64(0)
    miss = ctypes.c_int32(0)
    st = lib().orc_newton_solve(n, m, _p(C), beta, _p(u), _p(v), _p(r), _p(c), _p(lr),
                                float(eta), float(rho0), int(max_cg), int(max_levels),
                                _p(du), _p(dv), ctypes.byref(rho), ctypes.byref(it),
                                ctypes.byref(lev), ctypes.byref(np_), ctypes.byref(miss))
    return NewtonResult(du, dv, rho.value, it.value, lev.value, np_.value, int(st),
                        int(miss.value))


def chi_sinkhorn(C, beta, u, v, r, c, log_rP, eps_chi, max_iter=10000):
    C = _C(C); u = _d(u).copy(); v = _d(v).copy(); r = _d(r); c = _d(c)
    lr = _d(log_rP).copy()
    it = ctypes.c_int32(0)
    st = lib().orc_chi_sinkhorn(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v), _p(r),
                                _p(c), _p(lr), float(eps_chi), int(max_iter),
                                ctypes.byref(it))
    return u, v, lr, int(it.value), int(st)


def line_search(C, beta, u, v, grad_u, du, dv, max_backtrack=60, return_unresolved=False):
    C = _C(C); u = _d(u); v = _d(v); g = _d(grad_u); du = _d(du); dv = _d(dv)
    alpha = ctypes.c_double(0.0)
    lc = np.empty(C.shape[1])
    bt = ctypes.c_int32(0)
    unres = ctypes.c_int32(0)
    st = lib().orc_line_search(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v), _p(g),
                               _p(du), _p(dv), int(max_backtrack), ctypes.byref(alpha),
                               _p(lc), ctypes.byref(bt), ctypes.byref(unres))
    if return_unresolved:
        return alpha.value, lc, int(bt.value), int(st), int(unres.value)
    return alpha.value, lc, int(bt.value), int(st)


def default_opts(gamma_init=1.0 / 32.0, gamma_final=1e-3, tol=1e-6, **kw) -> Opts:
    o = Opts(gamma_init=gamma_init, gamma_final=gamma_final, tol=tol, p=1.5, q1=2.0,
             w_r=0.45, adaptive_q=1, adaptive_rho0=1, max_cg=1000, max_levels=30,
             max_backtrack=60, max_newton=200, max_sinkhorn=10000, max_mdot=500,
             projection=0)
    for k, val in kw.items():
        setattr(o, k, val)
    return o


def tnp(C, beta, u, v, r, c, eps, opts=None, rho0=0.0):
    C = _C(C); u = _d(u).copy(); v = _d(v).copy(); r = _d(r); c = _d(c)
    o = opts or default_opts()
    st = Stats()
    rho = ctypes.c_double(rho0)
    dmin = ctypes.c_double(0.0)
    status = lib().orc_tnp(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v), _p(r), _p(c),
                           float(eps), ctypes.byref(o), ctypes.byref(rho),
                           ctypes.byref(dmin), ctypes.byref(st))
    return u, v, dmin.value, rho.value, st.as_dict(), int(status)


def solve(C, r, c, opts=None, **kw):
    """MDOT + TruncatedNewtonProject. Returns (u, v, stats) with log-unit
    potentials at the final inverse temperature."""
    C = _C(C); r = _d(r); c = _d(c)
    o = opts or default_opts(**kw)
    n, m = C.shape
    u = np.empty(n); v = np.empty(m)
    st = Stats()
    status = lib().orc_solve(n, m, _p(C), _p(r), _p(c), ctypes.byref(o), _p(u), _p(v),
                             ctypes.byref(st))
    d = st.as_dict()
    d["status"] = int(status)
    return u, v, d


def round_plan(C, beta, u, v, r, c):
    C = _C(C); u = _d(u); v = _d(v); r = _d(r); c = _d(c)
    P = np.empty(C.shape)
    lib().orc_round(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v), _p(r), _p(c), _p(P))
    return P


# ---------------------------------------------------------------- traced solves

def _alloc_trace(n, m, cap_steps, cap_newton, potentials):
    bufs = {}
    tr = Trace(cap_steps=cap_steps, cap_newton=cap_newton)
    for k in STEP_FIELDS:
        a = np.zeros(cap_steps, dtype=np.int32 if k in INT_FIELDS else np.float64)
        bufs[k] = a
        setattr(tr, k, a.ctypes.data_as(_i32p if k in INT_FIELDS else _dp))
    for k in NEWTON_FIELDS:
        a = np.zeros(cap_newton, dtype=np.int32 if k in INT_FIELDS else np.float64)
        bufs[k] = a
        setattr(tr, k, a.ctypes.data_as(_i32p if k in INT_FIELDS else _dp))
    if potentials:
        bufs["u_proj"] = np.zeros((cap_steps, n))
        bufs["v_proj"] = np.zeros((cap_steps, m))
        tr.u_proj = _p(bufs["u_proj"])
        tr.v_proj = _p(bufs["v_proj"])
    return tr, bufs


def _trace_dict(tr, bufs):
    ns = min(tr.n_steps, tr.cap_steps)
    nk = min(tr.n_newton, tr.cap_newton)
    out = {"n_steps": tr.n_steps, "n_newton": tr.n_newton}
    for k in STEP_FIELDS:
        out[k] = bufs[k][:ns].copy()
    for k in NEWTON_FIELDS:
        out[k] = bufs[k][:nk].copy()
    if "u_proj" in bufs:
        out["u_proj"] = bufs["u_proj"][:ns].copy()
        out["v_proj"] = bufs["v_proj"][:ns].copy()
    return out


def _make_state(n, m, src=None):
    arrs = {k: np.zeros(n if k in ("u", "u_prev") else m) for k in ("u", "v", "u_prev", "v_prev")}
    st = State()
    if src is not None:
        st.t, st.beta, st.beta_prev = src["t"], src["beta"], src["beta_prev"]
        st.q, st.rho0 = src["q"], src["rho0"]
        for k in arrs:
            arrs[k][:] = src[k]
    for k, a in arrs.items():
        setattr(st, k, _p(a))
    return st, arrs


def solve_ex(C, r, c, opts=None, warm=None, resume=None, trace=True, potentials=False,
             cap_steps=512, cap_newton=4096, **kw):
    """MDOT + TruncatedNewtonProject with the step trace and the carried state.

    warm: (u0, v0) log-unit start at the first temperature; resume: a state
    dict from an earlier call. Returns (u, v, stats, trace dict or None, state dict)."""
    C = _C(C); r = _d(r); c = _d(c)
    o = opts or default_opts(**kw)
    n, m = C.shape
    u = np.zeros(n); v = np.zeros(m)
    if warm is not None:
        u[:] = warm[0]; v[:] = warm[1]
    st = Stats()
    tr, bufs = (_alloc_trace(n, m, cap_steps, cap_newton, potentials) if trace
                else (None, None))
    rs, _keep = _make_state(n, m, resume) if resume is not None else (None, None)
    so, sarr = _make_state(n, m)
    status = lib().orc_solve_ex(n, m, _p(C), _p(r), _p(c), ctypes.byref(o),
                                1 if warm is not None else 0,
                                ctypes.byref(rs) if rs is not None else None,
                                ctypes.byref(so), ctypes.byref(tr) if tr is not None else None,
                                _p(u), _p(v), ctypes.byref(st))
    d = st.as_dict()
    d["status"] = int(status)
    state = {"t": so.t, "beta": so.beta, "beta_prev": so.beta_prev, "q": so.q, "rho0": so.rho0,
             **{k: a.copy() for k, a in sarr.items()}}
    return u, v, d, (_trace_dict(tr, bufs) if tr is not None else None), state


def adjust_schedule(q, delta_min):
    return float(lib().orc_adjust_schedule(float(q), float(delta_min)))


def extrapolate(z, z_prev, beta_prev, beta, beta_next):
    z = _d(z).copy(); zp = _d(z_prev).copy()
    lib().orc_extrapolate(z.size, _p(z), _p(zp), float(beta_prev), float(beta), float(beta_next))
    return z, zp


def forcing_eta(gnorm, eps):
    return float(lib().orc_forcing_eta(float(gnorm), float(eps)))
