"""CPU emulation of the kernels' base-2 exponential and logarithm
(paper_1309_2710_amd/csrc/rkc_device.h: exp2_b31, exp2_sat, log2_pos), the
same operation sequence with correctly rounded FMAs, against 50-digit
references.  The rate constants of E:rxn-const are evaluated with these
functions, so their accuracy bounds what the source-term parity can reach."""
import math
import os
import random
import re
import struct
import sys
from fractions import Fraction

import mpmath as mp
import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1309_2710_amd", "csrc")
HDR = os.path.join(CSRC, "rkc_device.h")


def _exp_constants():
    """shift, ln2 and the ten polynomial coefficients as written in exp_k()."""
    src = open(HDR).read()
    body = src[src.index("constexpr ExpK exp_k()"):]
    body = body[body.index("return ExpK{") + len("return ExpK{"):body.index("}};")]
    nums = re.findall(r"0x[0-9a-fA-F.]+p[+-]?\d+|[-+]?\d+\.\d+(?:e[-+]?\d+)?", body)
    vals = [float.fromhex(x) if x.startswith("0x") else float(x) for x in nums]
    assert len(vals) == 12, vals
    return vals[0], vals[1], vals[2:]


SHIFT, LN2, C = _exp_constants()


def fma(a, b, c):
    if not (math.isfinite(a) and math.isfinite(b) and math.isfinite(c)):
        return a * b + c          # NaN and infinities: no rounding involved
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def ldexp(q, n):
    """v_ldexp_f64: q 2^n, rounded, saturating to 0 or inf."""
    if n > 2100:
        return math.copysign(math.inf, q)
    if n < -2200:
        return math.copysign(0.0, q)
    try:
        return math.ldexp(q, n)
    except OverflowError:
        return math.copysign(math.inf, q)


def exp2_frac(f):
    q = C[0]
    for c in C[1:]:
        q = fma(q, f, c)
    q = fma(q, f, LN2)
    return fma(q, f, 1.0)


def low_word_i32(t):
    lo = struct.unpack("<Q", struct.pack("<d", t))[0] & 0xFFFFFFFF
    return lo - (1 << 32) if lo >= (1 << 31) else lo


def exp2_b31(y):
    t = y + SHIFT
    n = t - SHIFT
    return ldexp(exp2_frac(y - n), low_word_i32(t))


def exp2_sat(y):
    t = y + SHIFT
    n = t - SHIFT
    # v_cvt_i32_f64: saturating, NaN gives 0
    ni = 0 if math.isnan(n) else int(max(min(n, 2 ** 31 - 1), -2 ** 31))
    return ldexp(exp2_frac(y - n), ni)


def log2_pos(x):
    m, e = math.frexp(x)
    l0 = float(np.log2(np.float32(m)))    # stands in for the hardware log2 seed
    d = fma(m, exp2_b31(-l0), -1.0)
    l1 = d * fma(d, fma(d, 1.0 / 3.0, -0.5), 1.0)
    return float(e) + fma(l1, 1.4426950408889634, l0)


def ulps(got, ref):
    ref = mp.mpf(ref)
    if ref == 0:
        return 0.0 if got == 0 else math.inf
    e = int(mp.floor(mp.log(abs(ref), 2)))
    ulp = mp.mpf(2) ** max(e - 52, -1074)
    return float(abs(mp.mpf(got) - ref) / ulp)


def test_coefficients_are_the_committed_fit():
    sys.path.insert(0, CSRC)
    try:
        import fit_exp_poly
    finally:
        sys.path.pop(0)
    cs, L, worst = fit_exp_poly.fit()
    assert cs == C
    assert L == LN2 == float(mp.log(2))
    assert worst < 3e-17
    assert SHIFT == 1.5 * 2.0 ** 52


def test_exp2_within_one_ulp():
    mp.mp.dps = 50
    rng = random.Random(7)
    ys = [rng.uniform(-1022.0, 1023.0) for _ in range(1500)] + \
         [rng.uniform(-60.0, 60.0) for _ in range(1500)] + \
         [k + s for k in range(-5, 6) for s in (-0.5, -0.25, 0.0, 0.25, 0.5)]
    worst = 0.0
    for y in ys:
        worst = max(worst, ulps(exp2_b31(y), mp.power(2, mp.mpf(y))))
    assert worst <= 1.0, worst
    assert exp2_b31(0.0) == 1.0 and exp2_b31(1.0) == 2.0 and exp2_b31(-1.0) == 0.5


def test_exp2_saturates_and_propagates_nan():
    for y in (-1100.0, -5e3, -2.0 ** 30):
        assert exp2_b31(y) == 0.0
        assert exp2_sat(y) == 0.0
    for y in (1025.0, 5e3, 2.0 ** 30):
        assert exp2_b31(y) == math.inf
        assert exp2_sat(y) == math.inf
    # the saturating form keeps going far beyond the int32 range
    for y in (-1e15, -3e9):
        assert exp2_sat(y) == 0.0
    for y in (1e15, 3e9):
        assert exp2_sat(y) == math.inf
    assert math.isnan(exp2_b31(math.nan)) and math.isnan(exp2_sat(math.nan))


def test_low_word_is_the_exponent_only_below_2_31():
    """Why the kernels bound 1/T in the Arrhenius factors: the low word of
    y + 1.5 2^52 is round(y) in two's complement while |y| < 2^31 and wraps
    beyond, where only the saturating form is right."""
    for y in (0.4, -0.6, 1074.5, -1e6, 2.0 ** 30, -(2.0 ** 30), 2.0 ** 31 - 1):
        assert low_word_i32(y + SHIFT) == round(y)
    assert low_word_i32(-3e9 + SHIFT) != -3000000000
    assert exp2_b31(-3e9) != 0.0          # wrapped: what the bound rules out


def test_log2_accuracy():
    mp.mp.dps = 50
    rng = random.Random(11)
    xs = [math.exp(rng.uniform(-700.0, 700.0)) for _ in range(1500)] + \
         [rng.uniform(200.0, 4000.0) for _ in range(500)] + \
         [1.0 + rng.uniform(-1e-3, 1e-3) for _ in range(300)]
    worst_rel = 0.0
    worst_abs = 0.0
    for x in xs:
        ref = mp.log(mp.mpf(x), 2)
        got = log2_pos(x)
        worst_abs = max(worst_abs, float(abs(mp.mpf(got) - ref)) / max(1.0, abs(float(ref))))
        if abs(ref) >= 1:
            worst_rel = max(worst_rel, ulps(got, ref))
    assert worst_rel <= 1.5, worst_rel
    assert worst_abs <= 2.0 ** -51, worst_abs
    assert log2_pos(1.0) == 0.0 and log2_pos(2.0) == 1.0 and log2_pos(0.5) == -1.0
