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
                ("levels", _i32), ("forcing_misses", _i32),
                ("passes_newton", ctypes.c_int64), ("passes_linesearch", ctypes.c_int64),
                ("passes_sinkhorn", ctypes.c_int64), ("passes_projection", ctypes.c_int64),
                ("final_beta", _f64), ("err_r", _f64), ("err_c", _f64),
                ("cost", _f64), ("dual_value", _f64), ("rho_last", _f64),
                ("delta_min_last", _f64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


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
                                               _dp, _i32, _dp, _dp, _i32p]),
            "orc_tnp": (ctypes.c_int, [_i64, _i64, _dp, _f64, _dp, _dp, _dp, _dp, _f64,
                                       ctypes.POINTER(Opts), _dp, _dp, ctypes.POINTER(Stats)]),
            "orc_solve": (ctypes.c_int, [_i64, _i64, _dp, _dp, _dp, ctypes.POINTER(Opts),
                                         _dp, _dp, ctypes.POINTER(Stats)]),
            "orc_round": (None, [_i64, _i64, _dp, _f64, _dp, _dp, _dp, _dp, _dp]),
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


def line_search(C, beta, u, v, grad_u, du, dv, max_backtrack=60):
    C = _C(C); u = _d(u); v = _d(v); g = _d(grad_u); du = _d(du); dv = _d(dv)
    alpha = ctypes.c_double(0.0)
    lc = np.empty(C.shape[1])
    bt = ctypes.c_int32(0)
    st = lib().orc_line_search(C.shape[0], C.shape[1], _p(C), beta, _p(u), _p(v), _p(g),
                               _p(du), _p(dv), int(max_backtrack), ctypes.byref(alpha),
                               _p(lc), ctypes.byref(bt))
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
