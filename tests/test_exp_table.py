"""The device exponential's table and reduction constants (lbfd_kernels.h,
exp_tab) against 60-digit decimal arithmetic: every entry 2^(j/256) is the
double nearest to the exact value, 256/ln 2 is the double nearest to it,
the head of ln 2/256 has at most 33 significant bits (so that n times it is
exact for |n| < 2^20) and head + tail is ln 2/256 to within the tail's own
rounding."""
import math
import os
import re
from decimal import Decimal, getcontext

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2304_05657_amd", "csrc", "lbfd_kernels.h")


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
