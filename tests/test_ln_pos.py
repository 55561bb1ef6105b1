"""The DI kernel's ln T (`ln_pos` in csrc/chemk_dev.h) checked on the CPU: its
constants are read from the source, its steps are replayed in float64 and
compared with the exact logarithm over the temperatures a cell can reach and
far beyond."""
import math
import os
import re
from decimal import Decimal, getcontext

import numpy as np

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2402_18858_amd", "csrc", "chemk_dev.h")


def _source():
    s = open(SRC).read()
    body = s[s.index("__device__ __forceinline__ double ln_pos"):]
    return body[:body.index("\n}\n")]


def _constants():
    body = _source()
    lo, hi = re.findall(r"fma\(de, ([0-9.eE+-]+),", body)
    terms = [int(v) for v in re.findall(r"1\.0 / (\d+)\.0", body)]
    return float(hi), float(lo), terms


def _ln_pos(x):
    hi, lo_c, terms = _constants()
    m, e = math.frexp(x)
    if m < 0.70710678118654752440:
        m, e = m + m, e - 1
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    p = 1.0 / terms[0]
    for t in terms[1:]:
        p = p * z + 1.0 / t
    lo = e * lo_c + 2.0 * (s * z * p)
    return e * hi + (lo + 2.0 * s)


def test_constants_split_ln2():
    getcontext().prec = 50
    hi, lo, terms = _constants()
    assert terms == [21, 19, 17, 15, 13, 11, 9, 7, 5, 3]
    ln2 = Decimal(2).ln()
    assert abs(Decimal(hi) + Decimal(lo) - ln2) < Decimal("3e-26")   # one ulp of lo
    # e * hi exact for any binary exponent: hi has 20+ trailing zero bits
    mant = int(hi * 2 ** 53)
    assert mant % (1 << 16) == 0


def test_within_a_few_ulp_of_log():
    rng = np.random.default_rng(3)
    xs = np.concatenate([np.linspace(200.0, 4000.0, 20001), 10.0 ** rng.uniform(-300, 300, 20000),
                         [1.0, 2.0, 0.5, math.sqrt(0.5), math.sqrt(2.0), 5e-324, 1.7e308]])
    worst = 0.0
    for x in xs:
        ref = math.log(x)
        got = _ln_pos(float(x))
        ulp = math.ulp(ref) if ref != 0.0 else 5e-324
        worst = max(worst, abs(got - ref) / ulp)
    # the replay rounds every product separately (the kernel fuses them): 3 ulp
    assert worst <= 3.0, worst
