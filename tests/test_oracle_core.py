"""Pins for the oracle's arithmetic core: rounding, ball operations, constants.

The oracle is only trusted after it agrees with things it does not compute
itself: the host's IEEE arithmetic (correctly rounded +, *, /, sqrt in binary64
and binary32/binary16 via numpy), an independent algorithm for pi (the
Gauss-Legendre AGM) and for ln 2 (sum 1/(k 2^k)), and the double-double
constants printed in the paper's tan listing (Appendix A: pi/2 and 2 pi as a
pair of binary64 numbers).
"""
import math
import random
import struct
from math import isqrt

import numpy as np
import pytest

from oracle import ball as B
from oracle.consts import pi, ln2, two_over_pi
from oracle.rounding import FORMATS, rn_dyadic, rn_ball

F64 = FORMATS["f64"]
F32 = FORMATS["f32"]
F16 = FORMATS["f16"]


def _rand_double(rng, lo_exp=-1074, hi_exp=1023):
    m = rng.getrandbits(52) | (1 << 52)
    e = rng.randint(lo_exp, hi_exp)
    return math.ldexp(m, e - 52) * rng.choice((1, -1))


def _exact(x):
    n, d = x.as_integer_ratio()
    return n, -(d.bit_length() - 1)


# --------------------------------------------------------------------------
# rounding core vs host IEEE operations
# --------------------------------------------------------------------------

def test_rn_products_match_ieee_binary64():
    rng = random.Random(1)
    checked = 0
    for _ in range(20000):
        a = _rand_double(rng, -560, 520)
        b = _rand_double(rng, -560, 520)
        ma, ea = _exact(a)
        mb, eb = _exact(b)
        got = rn_dyadic(ma * mb, ea + eb, F64)
        want = a * b
        assert got == want and math.copysign(1, got) == math.copysign(1, want), (a, b)
        checked += 1
    assert checked == 20000


def test_rn_products_into_subnormals_and_overflow():
    rng = random.Random(2)
    n_sub = 0
    for _ in range(20000):
        a = _rand_double(rng, -600, -400)
        b = _rand_double(rng, -700, -500)
        ma, ea = _exact(a)
        mb, eb = _exact(b)
        want = a * b
        got = rn_dyadic(ma * mb, ea + eb, F64)
        assert got == want and math.copysign(1, got) == math.copysign(1, want), (a, b)
        if want != 0 and abs(want) < 2.2250738585072014e-308:
            n_sub += 1
    assert n_sub > 1000
    for _ in range(5000):
        a = _rand_double(rng, 500, 1023)
        b = _rand_double(rng, 400, 1023)
        ma, ea = _exact(a)
        mb, eb = _exact(b)
        assert rn_dyadic(ma * mb, ea + eb, F64) == a * b


def test_rn_sums_match_ieee_binary64():
    rng = random.Random(3)
    for _ in range(20000):
        a = _rand_double(rng, -1074, 1000)
        b = _rand_double(rng, -1074, 1000) if rng.random() < 0.5 else \
            a * (1 + rng.uniform(-1e-10, 1e-10)) * rng.choice((1, -1))
        ma, ea = _exact(a)
        mb, eb = _exact(b)
        e = min(ea, eb)
        s = (ma << (ea - e)) + (mb << (eb - e))
        want = a + b
        got = rn_dyadic(s, e, F64)
        if s == 0:
            continue   # sign of an exact zero sum is not a rounding question
        assert got == want, (a, b)


def test_rn_binary32_and_binary16_products():
    rng = np.random.default_rng(4)
    a = (rng.standard_normal(20000) * np.exp2(rng.integers(-80, 60, 20000))).astype(np.float32)
    b = (rng.standard_normal(20000) * np.exp2(rng.integers(-80, 60, 20000))).astype(np.float32)
    prod = a * b                                   # IEEE binary32 RN
    for x, y, p in zip(a.tolist(), b.tolist(), prod.tolist()):
        mx, ex = _exact(x)
        my, ey = _exact(y)
        assert rn_dyadic(mx * my, ex + ey, F32) == p, (x, y)
    a16 = (rng.standard_normal(5000) * np.exp2(rng.integers(-10, 6, 5000))).astype(np.float16)
    b16 = (rng.standard_normal(5000) * np.exp2(rng.integers(-10, 6, 5000))).astype(np.float16)
    p16 = (a16.astype(np.float32) * b16.astype(np.float32)).astype(np.float16)
    for x, y, p in zip(a16.tolist(), b16.tolist(), p16.tolist()):
        mx, ex = _exact(x)
        my, ey = _exact(y)
        got = rn_dyadic(mx * my, ex + ey, F16)
        assert got == p or (math.isinf(got) and math.isinf(p)), (x, y)


def test_rn_ball_division_and_sqrt_match_ieee():
    rng = random.Random(5)
    for _ in range(5000):
        a = _rand_double(rng, -500, 500)
        b = _rand_double(rng, -500, 500)
        q = B.div(B.from_float(a), B.from_float(b), 120)
        assert rn_ball(q, F64) == a / b, (a, b)
        x = abs(a)
        s = B.sqrt(B.from_float(x), 120)
        assert rn_ball(s, F64) == math.sqrt(x), x


def test_ball_contains_exact_results():
    """Every ball operation must contain the exact rational result."""
    from fractions import Fraction
    rng = random.Random(6)

    def frac(b):
        return (Fraction(b.m - b.r) * Fraction(2) ** b.e,
                Fraction(b.m + b.r) * Fraction(2) ** b.e)

    for _ in range(3000):
        a = B.Ball(rng.getrandbits(90) - (1 << 89), rng.getrandbits(8), rng.randint(-200, 50))
        c = B.Ball(rng.getrandbits(70) | 1 << 69, rng.getrandbits(8), rng.randint(-200, 50))
        pa = Fraction(a.m) * Fraction(2) ** a.e + Fraction(rng.randint(-a.r, a.r)) * Fraction(2) ** a.e
        pc = Fraction(c.m) * Fraction(2) ** c.e + Fraction(rng.randint(-c.r, c.r)) * Fraction(2) ** c.e
        for op, val in ((B.add, pa + pc), (B.sub, pa - pc), (B.mul, pa * pc),
                        (B.div, pa / pc)):
            lo, hi = frac(op(a, c, 40))
            assert lo <= val <= hi
        if pc > 0:
            lo, hi = frac(B.sqrt(c, 40))
            assert lo * lo <= pc <= hi * hi


# --------------------------------------------------------------------------
# constants
# --------------------------------------------------------------------------

def _pi_agm(bits):
    """Gauss-Legendre AGM in fixed point (independent of Machin's formula)."""
    g = 64
    one = 1 << (bits + g)
    a = one
    b = isqrt(one * one // 2)
    t = one // 4
    p = 1
    for _ in range(int(math.log2(bits)) + 4):
        an = (a + b) // 2
        b = isqrt(a * b)
        t -= p * (a - an) ** 2 // one
        a = an
        p *= 2
    return (a + b) ** 2 // (4 * t), bits + g


def _ln2_other(bits):
    """ln 2 = sum_k 1 / (k 2^k) (a different series than the oracle's)."""
    g = 64
    one = 1 << (bits + g)
    s = 0
    k = 1
    while True:
        t = one // (k << k)
        if t == 0:
            break
        s += t
        k += 1
    return s, bits + g


def _agree(ball, m, frac_bits, bits):
    # |ball_mid - m * 2**-frac_bits| small compared with 2**-bits
    from fractions import Fraction
    mid = Fraction(ball.m) * Fraction(2) ** ball.e
    rad = Fraction(ball.r) * Fraction(2) ** ball.e
    other = Fraction(m, 1 << frac_bits)
    assert rad < Fraction(1, 1 << bits)
    assert abs(mid - other) < Fraction(1, 1 << bits)


def test_pi_two_algorithms_agree_to_1400_bits():
    m, fb = _pi_agm(1500)
    _agree(pi(1450), m, fb, 1420)


def test_ln2_two_series_agree():
    m, fb = _ln2_other(1200)
    _agree(ln2(1200), m, fb, 1150)


def test_constants_match_host_and_paper_double_double():
    assert rn_ball(pi(200), F64) == math.pi
    assert rn_ball(ln2(200), F64) == math.log(2)
    assert rn_ball(two_over_pi(200), F64) == 2 / math.pi
    # Appendix A, tan listing: pi/2 = 0x1.921fb54442d18p0 + 0x1.1a62633145c07p-54
    # and 2 pi = 0x1.921fb54442d18p2 + 0x1.1a62633145c07p-52 (hi, lo pairs).
    hp = B.scale2(pi(300), -1)
    hi = rn_ball(hp, F64)
    assert hi == float.fromhex("0x1.921fb54442d18p0")
    rest = B.sub(hp, B.from_float(hi), 300)
    assert rn_ball(rest, F64) == float.fromhex("0x1.1a62633145c07p-54")
    tp = B.scale2(pi(300), 1)
    hi2 = rn_ball(tp, F64)
    assert hi2 == float.fromhex("0x1.921fb54442d18p2")
    assert rn_ball(B.sub(tp, B.from_float(hi2), 300), F64) == \
        float.fromhex("0x1.1a62633145c07p-52")


def test_float32_constant_roundings():
    v = rn_ball(pi(100), F32)
    # float32(pi) from the host conversion of the double pi is correctly
    # rounded unless the double lies on a float midpoint (it does not)
    assert v == float(np.float32(np.float64(math.pi)))
    assert struct.pack("<f", v) == struct.pack("<f", 3.14159274101257324)


def test_rn_dyadic_bf16_matches_torch_conversion():
    """bf16 (p = 8, emin = -126): RN of binary32 values (random patterns over
    the whole range, bf16 subnormals, halfway cases, values just below and
    above the overflow threshold) equals torch's float32 -> bfloat16
    conversion, which rounds to nearest even."""
    import numpy as np
    import torch
    BF16 = FORMATS["bf16"]
    rng = np.random.default_rng(11)
    bits = [rng.integers(0, 0x7F800000, 20000, dtype=np.uint32)]
    bits.append(rng.integers(0, 0x00800000, 4000, dtype=np.uint32))       # f32 subnormals
    hw = rng.integers(0, 0x7F7F, 4000, dtype=np.uint32) << 16
    bits.append(hw | 0x8000)                                                 # exact halfway cases
    bits.append(hw | 0x7FFF)
    bits.append(hw | 0x8001)
    bits.append(np.arange(0x7F7F7FF0, 0x7F800000, dtype=np.uint32))         # overflow edge
    u = np.concatenate(bits)
    u = np.concatenate([u, u | np.uint32(0x80000000)])
    x = u.view(np.float32)
    want = torch.from_numpy(x.copy()).to(torch.bfloat16).to(torch.float64).numpy()
    n_inf = 0
    for xi, wi in zip(x.tolist(), want.tolist()):
        m, e = _exact(float(xi))
        got = rn_dyadic(m, e, BF16, zero_sign=-1 if math.copysign(1.0, xi) < 0 else 1)
        assert got == wi and math.copysign(1.0, got) == math.copysign(1.0, wi), (xi, got, wi)
        n_inf += math.isinf(got)
    assert n_inf > 0
