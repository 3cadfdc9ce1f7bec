"""Host check of the float64 exp used by the float64 kernel tiles (table-driven range
reduction, Tang's method): the arithmetic of exp_neg_tab, with the constants read from
the kernel source, is replayed here with correctly rounded fma (exact rationals) and
compared with a 50-digit exp.  Pins the accuracy stated for the float64 refinement
residuals; the GPU side is checked by test_fp64_kernel_entries_over_the_whole_exponent_range."""
import math
import os
import random
import re
from decimal import Decimal, getcontext
from fractions import Fraction

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2609_08136_amd", "csrc", "kmv_common.h")


def _constants():
    with open(SRC) as f:
        src = f.read()
    body = src[src.index("double exp_neg_tab("):]
    body = body[:body.index("\n}\n")]
    hexes = [float.fromhex(h) for h in re.findall(r"0x1\.[0-9a-f]+p[+-]?\d+", body)]
    assert len(hexes) == 3, hexes
    return hexes   # 64 / ln 2, head and tail of ln2 / 64


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))   # one correct rounding


def _exp_neg_tab(t, inv, head, tail, tab):
    t = max(t, -1100.0)
    kd = float(round(t * inv))                               # round half to even
    k = int(kd)
    r = _fma(-kd, head, t)
    r = _fma(-kd, tail, r)
    q = _fma(r, 1.0 / 120.0, 1.0 / 24.0)
    q = _fma(r, q, 1.0 / 6.0)
    q = _fma(r, q, 0.5)
    p = _fma(r * r, q, r)
    T = tab[k & 63]
    return math.ldexp(_fma(T, p, T), k >> 6)


def _table():
    getcontext().prec = 50
    ln2 = Decimal(2).ln()
    return [float((ln2 * j / 64).exp()) for j in range(64)]


def test_reduction_constants():
    getcontext().prec = 50
    inv, head, tail = _constants()
    L = Decimal(2).ln() / 64
    assert inv == float(1 / L)                                # 64/ln2 correctly rounded
    mant = Fraction(head).numerator
    while mant % 2 == 0:
        mant //= 2
    assert mant.bit_length() <= 36                            # k * head exact for |k| < 2^17
    assert abs(Decimal(head) + Decimal(tail) - L) <= Decimal(math.ulp(tail)) / 2   # tail correctly rounded


def test_table_exp_within_1p5_ulp():
    getcontext().prec = 50
    inv, head, tail = _constants()
    tab = _table()
    rng = random.Random(11)
    ts = [0.0, -0.0, 1e-12, -1e-300, -5e-324, -0.5 * math.log(2) / 64, -708.0, -709.78, -744.0, -745.1]
    ts += [-rng.uniform(0.0, 745.0) for _ in range(1500)]
    ts += [-math.exp(rng.uniform(-40.0, 6.0)) for _ in range(1500)]
    worst = 0.0
    for t in ts:
        got = _exp_neg_tab(t, inv, head, tail, tab)
        ref = Decimal(t).exp()
        if ref >= Decimal("2.2250738585072014e-308"):
            err = abs(Decimal(got) - ref) / Decimal(math.ulp(float(ref)))
            worst = max(worst, float(err))
            assert err <= Decimal("1.5"), (t, got, ref)
        else:                                                 # subnormal range
            assert abs(Decimal(got) - ref) <= Decimal(2) * Decimal(5e-324), (t, got)
    assert worst <= 1.5


def test_table_exp_limits():
    inv, head, tail = _constants()
    tab = _table()
    assert _exp_neg_tab(0.0, inv, head, tail, tab) == 1.0
    for t in (-746.0, -1100.0, -2000.0, -1e300, -math.inf):
        assert _exp_neg_tab(t, inv, head, tail, tab) == 0.0
