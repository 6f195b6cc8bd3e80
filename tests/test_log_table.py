"""The tables of the library's FP64 logarithm (made_log, made_kernels.h) and
its arithmetic, on the CPU: the committed header is what gen_log_table.py
writes, and the logarithm's steps, emulated with exact products (fma as one
rounding of the exact a b + c), are within one ulp of a 60-digit reference
logarithm on the thresholds' 2^-32 grid, next to 1 and across the exponent
range, with the two steps meant to be exact (the reduced argument and the
high part of the sum) exact."""
import decimal
import math
import os
import random
import re
import subprocess
import sys
from fractions import Fraction as Fr

import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2007_07379_amd", "csrc")


def tables():
    s = open(os.path.join(CSRC, "made_log_table.h")).read()

    def arr(name):
        body = s.split(name + "[256] = {")[1].split("};")[0]
        return [float.fromhex(x.strip()) if "0x" in x else int(x) for x in body.split(",")]

    hi = float.fromhex(re.search(r"MADE_LOG_LN2_HI = (\S+),", s).group(1))
    lo = float.fromhex(re.search(r"MADE_LOG_LN2_LO = (\S+);", s).group(1))
    return arr("MADE_LOG_G"), arr("MADE_LOG_K"), arr("MADE_LOG_TH"), arr("MADE_LOG_TL"), hi, lo


def test_header_is_the_generators_output():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_log_table.py")], check=True,
                         capture_output=True, text=True).stdout
    assert out == open(os.path.join(CSRC, "made_log_table.h")).read()


def emulated_log(x, G, K, TH, TL, LN2_HI, LN2_LO):
    """made_log's steps in order, each rounded as the GPU rounds it."""
    def fma(a, b, c):
        return float(Fr(a) * Fr(b) + Fr(c))

    m, e = math.frexp(x)
    m, e = 2.0 * m, e - 1  # m in [1, 2), exact
    j = int((m - 1.0) * 256.0)  # the top 8 fraction bits
    r = fma(m, G[j], -1.0)
    assert Fr(m) * Fr(G[j]) - 1 == Fr(r), "the reduced argument is exact"
    assert abs(r) <= 2.0 ** -8
    E = float(e + K[j])
    q = -0.125
    for c in (1.0 / 7.0, -1.0 / 6.0, 0.2, -0.25, 1.0 / 3.0, -0.5):
        q = fma(q, r, c)
    r2 = float(Fr(r) * Fr(r))
    lo = fma(r2, q, fma(E, LN2_LO, TL[j]))
    hi = fma(E, LN2_HI, TH[j])
    assert Fr(E) * Fr(LN2_HI) + Fr(TH[j]) == Fr(hi), "the high part is exact"
    return float(Fr(hi) + Fr(float(Fr(r) + Fr(lo))))


def test_emulated_log_within_one_ulp():
    G, K, TH, TL, LN2_HI, LN2_LO = tables()
    decimal.getcontext().prec = 60
    rng = random.Random(7)
    xs = [rng.randrange(1, 2 ** 32) * 2.0 ** -32 for _ in range(1500)]
    xs += [(2 ** 32 - rng.randrange(1, 2 ** 32)) * 2.0 ** -32 for _ in range(500)]
    xs += [1.0 - k * 2.0 ** -32 for k in range(1, 60)] + [1.0 + k * 2.0 ** -52 for k in range(1, 60)]
    xs += [1.0 - k * 2.0 ** -53 for k in range(1, 60)]
    xs += [2.0 ** rng.uniform(-1020, 1020) for _ in range(500)]
    xs += [2.0 ** -32, 0.5, 2.0, math.sqrt(2.0), 1.0 / math.sqrt(2.0), math.e, 1.0 / math.e]
    worst = 0.0
    for x in xs:
        y = emulated_log(x, G, K, TH, TL, LN2_HI, LN2_LO)
        ref = decimal.Decimal(x).ln()
        err = abs(decimal.Decimal(y) - ref) / decimal.Decimal(math.ulp(float(ref)))
        worst = max(worst, float(err))
    assert emulated_log(1.0, G, K, TH, TL, LN2_HI, LN2_LO) == 0.0
    assert worst <= 1.0, worst
