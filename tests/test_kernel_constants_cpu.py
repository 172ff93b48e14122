"""The FP64 exp of the streaming passes (table-driven, after Tang, ACM TOMS
15(2), 1989) takes its constants from csrc/eot_lanes.h: each table entry pair
must represent 2^(j/64) (hi rounded to nearest, hi + lo to ~2^-106), and the
reduction constants must be 64 / ln 2 and the hi / lo split of ln 2 / 64. Checked
against 60-digit decimal arithmetic; the function itself is covered by the FP64
GPU parity tests (1e-12 relative against the oracle)."""
import os
import re
from decimal import Decimal, getcontext

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2504_02067_amd", "csrc", "eot_lanes.h")


def _read():
    s = open(HDR).read()
    body = s[s.index("kExp2Tab64[128] = {") + len("kExp2Tab64[128] = {"):]
    body = body[:body.index("};")]
    tab = [float(t) for t in re.findall(r"[-+0-9.eE]+", body)]
    consts = dict((k, float(v)) for k, v in
                  re.findall(r"constexpr double (kInvLn2x64|kLn2d64Hi|kLn2d64Lo) = ([-+0-9.eE]+);", s))
    return tab, consts


def test_exp_table_entries():
    getcontext().prec = 60
    ln2 = Decimal(2).ln()
    tab, _ = _read()
    assert len(tab) == 128
    for j in range(64):
        exact = (ln2 * j / 64).exp()
        hi, lo = Decimal(tab[2 * j]), Decimal(tab[2 * j + 1])
        assert hi == Decimal(float(exact))                     # hi is the nearest double
        assert abs(hi + lo - exact) <= exact * Decimal(2) ** -104
        assert abs(lo) <= hi * Decimal(2) ** -53


def test_exp_reduction_constants():
    getcontext().prec = 60
    ln2 = Decimal(2).ln()
    _, c = _read()
    assert c["kInvLn2x64"] == float(64 / ln2)
    assert Decimal(c["kLn2d64Hi"]) == Decimal(float(ln2 / 64))
    assert abs(Decimal(c["kLn2d64Hi"]) + Decimal(c["kLn2d64Lo"]) - ln2 / 64) <= (ln2 / 64) * Decimal(2) ** -104
