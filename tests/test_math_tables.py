"""The device exponential and logarithm (lbfd_math.h, exp_tab and
log_tab) against 60-digit decimal arithmetic.  Tables: every entry 2^(j/256),
1/F_j and ln F_j (F_j = 1 + j/256) is the double nearest to the exact value.
Constants: 256/ln 2 and ln 2 are the nearest doubles, the head of ln 2/256
has at most 33 significant bits (n times it is exact for |n| < 2^20), and
each two-part constant is exact to within its tail's rounding.  Algorithms:
the three functions (with exp_scaled_tab, the exponential of a scaled
argument xs = x 256/ln 2) re-run step by step in Python doubles from the
header's own tables and constants (each fused multiply-add rounded once
through exact decimal arithmetic) stay within 1.5 ulp of the exact values
over the arguments the chemistry meets (log: 2 <= x <= 1e4 within 1.5 ulp,
and 1e-5 <= x < 2 within 1e-15 absolute; exp: -700 <= x <= 700)."""
import math
import os
import random
import re
import struct
from decimal import Decimal, getcontext

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2304_05657_amd", "csrc", "lbfd_math.h")


def _source():
    with open(SRC) as f:
        return f.read()


def _ln2():
    getcontext().prec = 60
    return Decimal(2).ln()


def test_table_entries_correctly_rounded():
    s = _source()
    n = int(re.search(r"constexpr int kExpTabN = (\d+);", s).group(1))
    body = s[s.index("kExp2Tab[kExpTabN] = {"):]
    body = body[:body.index("};")]
    vals = [float.fromhex(h) for h in re.findall(r"0x1\.[0-9a-f]+p[+-]\d+", body)]
    assert n == 256 and len(vals) == n
    ln2 = _ln2()
    for j, v in enumerate(vals):
        exact = (ln2 * j / n).exp()
        assert v == float(exact), j
        # and the neighbouring doubles are no nearer to it
        err = abs(Decimal(v) - exact)
        assert err <= abs(Decimal(math.nextafter(v, 2.0)) - exact)
        assert err <= abs(Decimal(math.nextafter(v, 0.0)) - exact)


def test_reduction_constants():
    s = _source()
    inv = float.fromhex(re.search(r"kInvLn2_256 = (0x[0-9a-fp.+-]+);", s).group(1))
    hi = float.fromhex(re.search(r"kLn2_256_hi = (0x[0-9a-fp.+-]+);", s).group(1))
    lo = float.fromhex(re.search(r"kLn2_256_lo = (0x[0-9a-fp.+-]+);", s).group(1))
    ln2 = _ln2()
    assert inv == float(256 / ln2)
    mant = int(hi.hex().split("p")[0].replace("0x1.", ""), 16)
    assert mant & ((1 << 20) - 1) == 0  # 52 - 20 = 32 fraction bits at most
    assert lo == float(ln2 / 256 - Decimal(hi))
    # within half an ulp of the tail (2^-93 for a tail in [2^-41, 2^-40))
    assert abs(Decimal(hi) + Decimal(lo) - ln2 / 256) <= Decimal(2) ** -94


def _fma(a, b, c):
    return float(Decimal(a) * Decimal(b) + Decimal(c))


def _table(s, decl):
    body = s[s.index(decl):]
    body = body[body.index("{") + 1:body.index("};")]
    return [float.fromhex(t.strip()) if "x" in t else float(t) for t in body.split(",") if t.strip()]


def _const(s, name):
    return float.fromhex(re.search(name + r" = (0x[0-9a-fp.+-]+);", s).group(1))


def test_log_table_entries_correctly_rounded():
    s = _source()
    tab = _table(s, "kLogTab[2 * kLogTabN] = {")
    assert len(tab) == 512
    getcontext().prec = 60
    for j in range(256):
        F = 1 + j / 256
        assert tab[2 * j] == 1.0 / F  # IEEE division rounds to nearest
        assert tab[2 * j + 1] == float(Decimal(F).ln()), j
    ln2 = _ln2()
    assert _const(s, "kLn2") == float(ln2)
    assert _const(s, "kLn2_lo") == float(ln2 - Decimal(_const(s, "kLn2")))


def _log_tab(x, tab, ln2, ln2_lo):
    bits = struct.unpack("<Q", struct.pack("<d", x))[0]
    hi, lo = bits >> 32, bits & 0xFFFFFFFF
    j = (hi >> 12) & 0xFF
    m = struct.unpack("<d", struct.pack("<Q", (((hi & 0x000FFFFF) | 0x3FF00000) << 32) | lo))[0]
    F = struct.unpack("<d", struct.pack("<Q", ((hi & 0x000FF000) | 0x3FF00000) << 32))[0]
    r = (m - F) * tab[2 * j]
    p = _fma(r, -1.0 / 6.0, 0.2)
    p = _fma(r, p, -0.25)
    p = _fma(r, p, 1.0 / 3.0)
    p = _fma(r, p, -0.5)
    l1p = _fma(r * r, p, r)
    e = float((hi >> 20) - 1023)
    return _fma(e, ln2, tab[2 * j + 1]) + _fma(e, ln2_lo, l1p)


def _exp_tab(x, tab, inv, hi, lo):
    x = min(max(x, -1000.0), 1000.0)
    n = float(round(x * inv))  # round half to even, as rint
    r = _fma(-n, lo, _fma(-n, hi, x))
    ni = int(n)
    p = _fma(r, 1.0 / 24.0, 1.0 / 6.0)
    p = _fma(r, p, 0.5)
    p = _fma(r, p, 1.0)
    p *= r
    t = tab[ni & 255]
    return math.ldexp(_fma(t, p, t), ni >> 8)


def test_log_and_exp_algorithms():
    s = _source()
    ltab = _table(s, "kLogTab[2 * kLogTabN] = {")
    etab = _table(s, "kExp2Tab[kExpTabN] = {")
    ln2, ln2_lo = _const(s, "kLn2"), _const(s, "kLn2_lo")
    inv, hi, lo = _const(s, "kInvLn2_256"), _const(s, "kLn2_256_hi"), _const(s, "kLn2_256_lo")
    getcontext().prec = 60
    rng = random.Random(7)
    xs = [rng.uniform(2.0, 1e4) for _ in range(1500)] + [2.0, 2.0 ** 10, 300.0, 1e4]
    for x in xs:
        exact = Decimal(x).ln()
        assert abs(Decimal(_log_tab(x, ltab, ln2, ln2_lo)) - exact) <= Decimal(1.5 * math.ulp(float(exact))), x
    for x in [rng.uniform(1e-5, 2.0) for _ in range(800)] + [1.0, 0.5, 1.0 - 2.0 ** -30]:
        exact = Decimal(x).ln()
        assert abs(Decimal(_log_tab(x, ltab, ln2, ln2_lo)) - exact) <= Decimal("1e-15"), x
    for x in [rng.uniform(-700.0, 700.0) for _ in range(1500)] + [0.0, -1.0, 1e-20, -745.0 + 1.0]:
        exact = Decimal(x).exp()
        assert abs(Decimal(_exp_tab(x, etab, inv, hi, lo)) - exact) <= Decimal(1.5 * math.ulp(float(exact))), x


def _exp_scaled_tab(xs, tab, k):
    xs = max(xs, -370000.0)
    n = float(round(xs))
    sr = xs - n
    p = _fma(sr, k[3], k[2])
    p = _fma(sr, p, k[1])
    p = _fma(sr, p, k[0])
    p *= sr
    ni = int(n)
    t = tab[ni & 255]
    return math.ldexp(_fma(t, p, t), ni >> 8)


def test_scaled_exponential():
    s = _source()
    etab = _table(s, "kExp2Tab[kExpTabN] = {")
    getcontext().prec = 60
    k1 = _ln2() / 256
    k = [_const(s, "k%d" % i) for i in (1, 2, 3, 4)]
    for i, f in enumerate((1, 2, 6, 24)):
        assert k[i] == float(k1 ** (i + 1) / f)
    assert float.fromhex("0x1.71547652b82fep+8") == float(1 / k1)  # the scale the host applies
    rng = random.Random(11)
    for x in [rng.uniform(-700.0, 700.0) for _ in range(1500)] + [0.0, -1.0, 1e-20]:
        xs = x * float(1 / k1)
        exact = (Decimal(xs) * k1).exp()  # exp of the argument as given
        assert abs(Decimal(_exp_scaled_tab(xs, etab, k)) - exact) <= Decimal(1.5 * math.ulp(float(exact))), x
    assert _exp_scaled_tab(-1e300, etab, k) == 0.0
