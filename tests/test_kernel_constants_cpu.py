"""The FP64 exp of the streaming passes (exp_tab256 in csrc/eot_lanes.h:
table-driven after Tang, ACM TOMS 15(2), 1989, with 256 entries). Its
constants are read from the header and checked against 60-digit decimal
arithmetic: each table pair must represent 2^(j/256) (hi rounded to nearest,
hi + lo to ~2^-106), the reduction constants must be 256 / ln 2 and the hi / lo
split of ln 2 / 256, and the rounding constant 1.5 * 2^52. The algorithm itself
is then replayed on the CPU step by step (every fma rounded once, through exact
rational arithmetic) and its error measured against e^x to 40 digits: at most
0.9 ulp, with the special values the passes rely on. The GPU parity tests cover
the compiled function (1e-12 relative against the oracle)."""
import math
import os
import re
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2504_02067_amd", "csrc", "eot_lanes.h")


def _read():
    s = open(HDR).read()
    key = "kExp2Tab256[512] = {"
    body = s[s.index(key) + len(key):]
    body = body[:body.index("};")]
    tab = [float(t) for t in re.findall(r"[-+0-9.eE]+", body)]
    consts = dict((k, float(v)) for k, v in
                  re.findall(r"constexpr double (kExpRound|kExpInvLn2x256|kExpLn2d256Hi|kExpLn2d256Lo) = "
                             r"([-+0-9.eE]+);", s))
    return tab, consts


def test_exp_table_entries():
    getcontext().prec = 60
    ln2 = Decimal(2).ln()
    tab, _ = _read()
    assert len(tab) == 512
    for j in range(256):
        exact = (ln2 * j / 256).exp()
        hi, lo = Decimal(tab[2 * j]), Decimal(tab[2 * j + 1])
        assert hi == Decimal(float(exact))                     # hi is the nearest double
        assert abs(hi + lo - exact) <= exact * Decimal(2) ** -104
        assert abs(lo) <= hi * Decimal(2) ** -53


def test_exp_constants():
    getcontext().prec = 60
    ln2 = Decimal(2).ln()
    _, c = _read()
    assert c["kExpRound"] == 1.5 * 2.0 ** 52
    assert c["kExpInvLn2x256"] == float(256 / ln2)
    assert Decimal(c["kExpLn2d256Hi"]) == Decimal(float(ln2 / 256))
    assert abs(Decimal(c["kExpLn2d256Hi"]) + Decimal(c["kExpLn2d256Lo"]) - ln2 / 256) \
        <= (ln2 / 256) * Decimal(2) ** -104


def _fma(a, b, c):
    """a * b + c rounded once (exact rational arithmetic, then one rounding)."""
    if not all(math.isfinite(x) for x in (a, b, c)):
        return a * b + c
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def _exp_replay(x, tab, c):
    """exp_tab256, step by step, in the device's order of operations."""
    x = max(min(x, 710.0), -1100.0) if not math.isnan(x) else 710.0    # fmin(NaN, .) = 710
    kd = _fma(x, c["kExpInvLn2x256"], c["kExpRound"])
    kf = kd - c["kExpRound"]
    bits = np.array([kd], dtype=np.float64).view(np.uint64)[0]
    k = int(np.array([bits & np.uint64(0xFFFFFFFF)], dtype=np.uint32).view(np.int32)[0])
    r = _fma(-kf, c["kExpLn2d256Lo"], _fma(-kf, c["kExpLn2d256Hi"], x))
    t = _fma(_fma(1.0 / 24.0, r, 1.0 / 6.0), r, 0.5)
    s = _fma(r * r, t, r)
    th, tl = tab[2 * (k & 255)], tab[2 * (k & 255) + 1]
    v = th + _fma(th, s, tl)
    try:
        return math.ldexp(v, k >> 8)
    except OverflowError:
        return math.inf


def test_exp_replay_error_bound():
    getcontext().prec = 40
    tab, c = _read()
    rng = np.random.default_rng(7)
    ln2 = math.log(2.0)
    xs = np.concatenate([rng.uniform(-3.0, 3.0, 1500), rng.uniform(-708.0, 709.7, 1500),
                         np.arange(-40, 41) * ln2 / 256.0,               # table points
                         (np.arange(-40, 41) + 0.5) * ln2 / 256.0])      # |r| at its bound
    worst = 0.0
    for x in xs:
        x = float(x)
        got = _exp_replay(x, tab, c)
        ref = Decimal(x).exp()
        ulp = Decimal(2) ** (math.frexp(float(ref))[1] - 53)
        worst = max(worst, float(abs(Decimal(got) - ref) / ulp))
    assert worst <= 0.9, worst


def test_exp_replay_special_values():
    tab, c = _read()
    assert _exp_replay(0.0, tab, c) == 1.0
    assert _exp_replay(-0.0, tab, c) == 1.0
    assert _exp_replay(math.log(2.0), tab, c) == 2.0
    assert _exp_replay(-math.inf, tab, c) == 0.0
    assert _exp_replay(-1e300, tab, c) == 0.0
    assert _exp_replay(-746.0, tab, c) == 0.0
    assert _exp_replay(-744.5, tab, c) > 0.0                  # subnormal, not flushed
    assert _exp_replay(709.79, tab, c) == math.inf
    assert _exp_replay(709.78, tab, c) == math.exp(709.78)
    assert _exp_replay(math.inf, tab, c) == math.inf
    assert _exp_replay(math.nan, tab, c) == math.inf          # non-finite, as the checks need
