"""Pins for the oracle's functions against things it does not compute itself.

* Annex F special values against the host C library (numpy calls glibc, whose
  special-value behaviour follows C99 Annex F).
* Correct rounding against mpmath evaluated at 400 bits (an independent
  multiprecision implementation), on regular grids, random bit patterns and
  huge trigonometric arguments (the paper's tester uses regular intervals,
  arguments near multiples of pi/2 and random bit patterns; Section 6).
* binary32 results against glibc's binary64 functions rounded to binary32:
  where they disagree, the binary64 value must lie within two binary64 ulps
  of a binary32 rounding midpoint (double rounding), which is the only way a
  correctly rounded binary32 result can differ from it.
* Exact cases: pow(x, 1/2) = sqrt(x), pow(x, 2) = x*x, pow(x, -1) = 1/x (IEEE
  operations are correctly rounded), exp2 and log2 at powers of two, fmod and
  remainder against the host's exact fmod/remainder, and the paper's worked
  remainder example fmod(1e40, 0.75) = 0.25 (Section 5, "FP Remainder").
* Identities evaluated on the oracle's balls: sin^2 + cos^2 = 1,
  cosh^2 - sinh^2 = 1, exp(log x) = x.
"""
import math
import os
import random
import warnings
import zlib

import mpmath
import numpy as np
import pytest

from oracle import evaluate, evaluate1
from oracle import ball as B
from oracle.elementary import exp_ball, log_ball, sincos_reduced, sin_cos_ball, sinh_cosh_small
from oracle.rounding import FORMATS, rn_ball

warnings.simplefilter("ignore", RuntimeWarning)

SPECIALS = [0.0, -0.0, math.inf, -math.inf, math.nan, 1.0, -1.0, 0.5, -0.5,
            2.0, -2.0, 3.0, -3.0, 2.5, -2.5, 5e-324, -5e-324, 1e300, -1e300]

NP_UNARY = {"sin": np.sin, "cos": np.cos, "tan": np.tan, "exp": np.exp,
            "exp2": np.exp2, "log": np.log, "log2": np.log2, "sinh": np.sinh,
            "cosh": np.cosh, "tanh": np.tanh, "asin": np.arcsin, "acos": np.arccos,
            "atan": np.arctan, "log10": np.log10, "exp10": lambda x: np.power(10.0, x),
            "expm1": np.expm1, "log1p": np.log1p, "cbrt": np.cbrt, "asinh": np.arcsinh,
            "acosh": np.arccosh, "atanh": np.arctanh,
            "erf": np.vectorize(math.erf, otypes=[np.float64]),
            "erfc": np.vectorize(math.erfc, otypes=[np.float64])}


def same(a, b):
    if math.isnan(a) or math.isnan(b):
        return math.isnan(a) and math.isnan(b)
    return a == b and math.copysign(1, a) == math.copysign(1, b)


# --------------------------------------------------------------------------
# Annex F
# --------------------------------------------------------------------------

@pytest.mark.parametrize("fn", sorted(NP_UNARY))
def test_unary_specials_match_host_libm(fn):
    for x in [0.0, -0.0, math.inf, -math.inf, math.nan, 1.0, -1.0]:
        if fn in ("erf", "erfc") and abs(x) == 1.0:
            continue       # not special there, and the host's erfc(-1) is 1 ulp off
        got = evaluate1(fn, "f64", x)[0]
        want = float(NP_UNARY[fn](np.float64(x)))
        assert same(got, want), (fn, x, got, want)


def _is_special(v):
    return v == 0 or not math.isfinite(v)


def test_pow_atan2_fmod_remainder_special_grid_matches_host_libm():
    # only the Annex F cases: a special argument or a special result (numpy's
    # own atan2 is not correctly rounded for ordinary arguments)
    for x in SPECIALS:
        for y in SPECIALS:
            if not (_is_special(x) or _is_special(y) or x in (1.0, -1.0)):
                continue
            for fn, host in (("pow", np.power), ("atan2", np.arctan2),
                             ("fmod", np.fmod), ("remainder", None)):
                got = evaluate1(fn, "f64", x, y)[0]
                if host is None:
                    try:
                        want = math.remainder(x, y)
                    except ValueError:
                        want = math.nan
                else:
                    want = float(host(np.float64(x), np.float64(y)))
                if fn == "atan2" and math.isfinite(want) and want != 0:
                    want = math.atan2(x, y)     # glibc's atan2
                assert same(got, want), (fn, x, y, got, want)


def test_binary32_specials_match_host_libm():
    for x in SPECIALS:
        xf = float(np.float32(x))
        for fn, f in NP_UNARY.items():
            got = evaluate1(fn, "f32", xf)[0]
            want = float(f(np.float32(xf)))
            if math.isnan(want) or math.isinf(want) or want == 0.0:
                assert same(got, want), (fn, xf)
        for y in SPECIALS:
            yf = float(np.float32(y))
            for fn, host in (("pow", np.power), ("atan2", np.arctan2)):
                got = evaluate1(fn, "f32", xf, yf)[0]
                want = float(host(np.float32(xf), np.float32(yf)))
                if math.isnan(want) or math.isinf(want) or want == 0.0 or \
                        not math.isfinite(xf) or not math.isfinite(yf) or xf == 0 or yf == 0:
                    assert same(got, want), (fn, xf, yf, got, want)


# --------------------------------------------------------------------------
# correct rounding vs mpmath at 400 bits
# --------------------------------------------------------------------------

MP = {"sin": mpmath.sin, "cos": mpmath.cos, "tan": mpmath.tan,
      "exp": mpmath.exp, "exp2": lambda x: mpmath.power(2, x),
      "log": mpmath.log, "log2": lambda x: mpmath.log(x, 2),
      "sinh": mpmath.sinh, "cosh": mpmath.cosh, "tanh": mpmath.tanh,
      "asin": mpmath.asin, "acos": mpmath.acos, "atan": mpmath.atan,
      "log10": mpmath.log10, "exp10": lambda x: mpmath.power(10, x),
      "expm1": mpmath.expm1, "log1p": mpmath.log1p,
      "cbrt": lambda x: mpmath.sign(x) * mpmath.cbrt(abs(x)),   # the real root
      "asinh": mpmath.asinh, "acosh": mpmath.acosh, "atanh": mpmath.atanh,
      "erf": mpmath.erf, "erfc": mpmath.erfc}


def _mp_f64(fn, x, y=None):
    with mpmath.workprec(400):
        if fn == "pow":
            v = mpmath.power(mpmath.mpf(x), mpmath.mpf(y))
        elif fn == "atan2":
            v = mpmath.atan2(mpmath.mpf(x), mpmath.mpf(y))
        elif fn == "hypot":
            v = mpmath.hypot(mpmath.mpf(x), mpmath.mpf(y))
        else:
            v = MP[fn](mpmath.mpf(x))
        return v


def _to_f64(v):
    # mpmath's float() rounds to nearest in 53 bits; beyond the double range
    # it gives inf.  Below 2^-1022 it would round twice (to 53 bits, then to
    # the subnormal grid), so there the value is rounded once to a multiple
    # of 2^-1074 (mpmath's nint: ties to even).
    if v != 0 and abs(v) < mpmath.mpf(2) ** -1022:
        with mpmath.workprec(600):
            n = mpmath.nint(v * mpmath.mpf(2) ** 1074)
        return math.copysign(float(n) * 2.0 ** -1074, float(v)) if n == 0 else float(n) * 2.0 ** -1074
    try:
        return float(v)
    except OverflowError:
        return math.inf if v > 0 else -math.inf


def _inputs(fn, rng, n):
    xs = []
    for _ in range(n):
        c = rng.random()
        if fn in ("log", "log2", "log10"):
            xs.append(abs(_rand_bits(rng)) if c < 0.5 else rng.uniform(0, 1000))
        elif fn == "log1p":
            if c < 0.3:
                xs.append(rng.uniform(-1, 1))
            elif c < 0.6:
                xs.append(math.copysign(10 ** rng.uniform(-310, 0), rng.random() - 0.5))
            else:
                xs.append(abs(_rand_bits(rng)))
        elif fn == "acosh":
            xs.append(1 + 10 ** rng.uniform(-16, 0) if c < 0.4 else abs(_rand_bits(rng)) + 1.0)
        elif fn == "atanh":
            xs.append(math.copysign(1 - 10 ** rng.uniform(-16, 0), rng.random() - 0.5) if c < 0.4
                      else math.copysign(10 ** rng.uniform(-310, 0), rng.random() - 0.5))
        elif fn in ("erf", "erfc"):
            if c < 0.5:
                xs.append(rng.uniform(-6, 6))
            elif c < 0.8:
                xs.append(rng.uniform(-1, 28))
            else:
                xs.append(math.copysign(10 ** rng.uniform(-310, 0), rng.random() - 0.5))
        elif fn in ("exp10", "expm1"):
            lim = 330 if fn == "exp10" else 760
            xs.append(rng.uniform(-lim, lim) if c < 0.5 else
                      math.copysign(10 ** rng.uniform(-300, 3), rng.random() - 0.5))
        elif fn in ("asin", "acos"):
            if c < 0.4:
                xs.append(rng.uniform(-1, 1))
            elif c < 0.7:                 # within 10^-16 .. 1 of +-1
                xs.append(math.copysign(1 - 10 ** rng.uniform(-16, 0), rng.random() - 0.5))
            else:
                xs.append(math.copysign(10 ** rng.uniform(-310, 0), rng.random() - 0.5))
        elif fn in ("exp", "exp2", "sinh", "cosh", "tanh"):
            lim = 1100 if fn == "exp2" else 760
            xs.append(rng.uniform(-lim, lim) if c < 0.5 else
                      math.copysign(10 ** rng.uniform(-300, 3), rng.random() - 0.5))
        else:
            xs.append(rng.uniform(-10, 10) if c < 0.4 else _rand_bits(rng))
    return [x for x in xs if math.isfinite(x) and x != 0]


def _rand_bits(rng):
    import struct
    return struct.unpack("<d", rng.getrandbits(64).to_bytes(8, "little"))[0]


@pytest.mark.parametrize("fn", sorted(MP))
def test_unary_correct_rounding_vs_mpmath(fn):
    rng = random.Random(zlib.crc32(fn.encode()) & 0xffff)
    for x in _inputs(fn, rng, 250):
        got, hi, lo = evaluate1(fn, "f64", x)
        v = _mp_f64(fn, x)
        want = _to_f64(v)
        assert same(got, want), (fn, x.hex(), got, want)
        if math.isfinite(got) and got != 0 and abs(got) > 1e-290:
            with mpmath.workprec(400):
                err = abs((mpmath.mpf(hi) + mpmath.mpf(lo)) - v) / abs(v)
            assert err < mpmath.mpf(2) ** -100, (fn, x)


def test_trig_huge_and_near_multiples_of_half_pi_vs_mpmath():
    rng = random.Random(11)
    xs = [6381956970095103.0 * 2.0 ** 797, 1e22, 1e300, 1.7976931348623157e308,
          5.319372648326541e255, 2.0 ** 1000]
    # doubles nearest to k pi/2 for assorted k (the reduction's hard cases)
    with mpmath.workprec(300):
        for k in [1, 2, 3, 7, 11, 355, 710, 1e6, 123456789, 2 ** 40 + 3, 2 ** 50 + 1]:
            xs.append(float(mpmath.mpf(k) * mpmath.pi / 2))
    xs += [math.ldexp(rng.random(), rng.randint(10, 1023)) for _ in range(60)]
    for fn in ("sin", "cos", "tan"):
        for x in xs:
            got = evaluate1(fn, "f64", x)[0]
            with mpmath.workprec(2600):
                v = MP[fn](mpmath.mpf(x))
            assert same(got, _to_f64(v)), (fn, x)


def test_pow_atan2_correct_rounding_vs_mpmath():
    rng = random.Random(7)
    for _ in range(300):
        x = rng.uniform(0, 30) if rng.random() < 0.6 else abs(_rand_bits(rng))
        y = rng.uniform(-30, 30) if rng.random() < 0.6 else rng.uniform(-1e3, 1e3)
        if not (math.isfinite(x) and x > 0):
            continue
        got = evaluate1("pow", "f64", x, y)[0]
        want = _to_f64(_mp_f64("pow", x, y))
        if want != 0 and abs(want) < 2.2250738585072014e-308:
            with mpmath.workprec(400):
                want = float(mpmath.mpf(_mp_f64("pow", x, y)))
        assert same(got, want), ("pow", x, y, got, want)
    for _ in range(300):
        y = _rand_bits(rng) if rng.random() < 0.5 else rng.uniform(-10, 10)
        x = _rand_bits(rng) if rng.random() < 0.5 else rng.uniform(-10, 10)
        if not (math.isfinite(x) and math.isfinite(y)) or x == 0 or y == 0:
            continue
        got = evaluate1("atan2", "f64", y, x)[0]
        want = _to_f64(_mp_f64("atan2", y, x))
        assert same(got, want), ("atan2", y, x, got, want)


def test_negative_base_integer_exponent_sign():
    for x, y in ((-2.0, 3.0), (-2.0, 4.0), (-1.5, 7.0), (-3.0, -3.0), (-0.7, 101.0)):
        got = evaluate1("pow", "f64", x, y)[0]
        with mpmath.workprec(400):
            want = float(mpmath.power(mpmath.mpf(x), mpmath.mpf(y)))
        assert same(got, want), (x, y)


# --------------------------------------------------------------------------
# binary32 against glibc binary64 rounded once more
# --------------------------------------------------------------------------

def _midpoint_distance_in_dulps(d):
    """Distance of the binary64 value d to the nearest binary32 rounding
    midpoint, in binary64 ulps of d."""
    f = np.float32(d)
    lo = np.nextafter(f, np.float32(-np.inf))
    hi = np.nextafter(f, np.float32(np.inf))
    mids = [(float(f) + float(lo)) / 2, (float(f) + float(hi)) / 2]
    u = math.ulp(d)
    return min(abs(d - m) for m in mids) / u


@pytest.mark.parametrize("fn", ["sin", "cos", "tan", "exp", "log", "exp2", "log2",
                                "sinh", "cosh", "tanh", "asin", "acos", "atan",
                                "log10", "exp10", "expm1", "log1p", "cbrt", "asinh",
                                "acosh", "atanh", "erf", "erfc"])
def test_binary32_vs_glibc_double_rounded(fn):
    # a strided sweep over all positive and negative binary32 bit patterns
    stride = 1 << 16
    bits = np.arange(0, 1 << 32, stride, dtype=np.uint64) + 12345
    xs = bits.astype(np.uint32).view(np.float32)
    xs = xs[np.isfinite(xs)]
    rn, _, _ = evaluate(fn, "f32", xs)
    d = NP_UNARY[fn](xs.astype(np.float64))
    f = d.astype(np.float32).astype(np.float64)
    bad = ~((rn == f) | (np.isnan(rn) & np.isnan(f)))
    for i in np.nonzero(bad)[0]:
        assert math.isfinite(d[i]) and _midpoint_distance_in_dulps(d[i]) <= 2.0, \
            (fn, float(xs[i]), rn[i], f[i])
    assert bad.sum() <= max(2, len(xs) // 1000)


# --------------------------------------------------------------------------
# exact cases
# --------------------------------------------------------------------------

def test_pow_exact_cases_against_ieee_operations():
    rng = random.Random(9)
    for _ in range(2000):
        x = abs(_rand_bits(rng))
        if not math.isfinite(x) or x == 0:
            continue
        assert evaluate1("pow", "f64", x, 0.5)[0] == math.sqrt(x), x
        assert evaluate1("pow", "f64", x, -1.0)[0] == 1.0 / x, x
        assert evaluate1("pow", "f64", x, 1.0)[0] == x
        sq = x * x
        assert same(evaluate1("pow", "f64", x, 2.0)[0], sq), x
        assert same(evaluate1("pow", "f64", -x, 2.0)[0], sq), x
    for n in range(-1080, 1030, 7):
        want = math.inf if n >= 1024 else (math.ldexp(1.0, n) if n > -1075 else 0.0)
        assert evaluate1("pow", "f64", 2.0, float(n))[0] == want
        assert evaluate1("exp2", "f64", float(n))[0] == want
    for n in range(-1074, 1024, 5):
        assert evaluate1("log2", "f64", 2.0 ** n)[0] == float(n)
    # small odd bases: exact products
    for b in (3.0, 5.0, 7.0, 0.75, 1.5):
        for k in range(1, 40):
            assert evaluate1("pow", "f64", b, float(k))[0] == float(mpmath.mpf(b) ** k)


def test_fmod_remainder_exact_against_host():
    rng = random.Random(10)
    for _ in range(20000):
        x = _rand_bits(rng)
        y = _rand_bits(rng) if rng.random() < 0.7 else rng.uniform(-10, 10)
        if not (math.isfinite(x) and math.isfinite(y)) or y == 0:
            continue
        assert same(evaluate1("fmod", "f64", x, y)[0], math.fmod(x, y)), (x, y)
        assert same(evaluate1("remainder", "f64", x, y)[0], math.remainder(x, y)), (x, y)


def test_fmod_paper_worked_example():
    # Section 5, "FP Remainder": fmod(1e40, 0.75); the exact answer is 0.25
    assert evaluate1("fmod", "f64", 1e40, 0.75)[0] == 0.25


def test_atan2_quadrant_constants():
    q = evaluate1("atan2", "f64", 1.0, 1.0)[0]
    assert q == math.pi / 4
    for y in (1e-300, 3.0, 1e300):
        assert evaluate1("atan2", "f64", y, y)[0] == math.pi / 4
        assert evaluate1("atan2", "f64", y, 0.0)[0] == math.pi / 2
        assert evaluate1("atan2", "f64", -y, -y)[0] == -3 * math.pi / 4


# --------------------------------------------------------------------------
# identities on balls
# --------------------------------------------------------------------------

def _contains_one(b):
    lo, hi, e = b.lo_hi()
    return lo * 2 ** e <= 1 <= hi * 2 ** e if e >= 0 else (lo <= (1 << -e) <= hi)


def test_inverse_trig_identities_on_balls():
    """asin x + acos x = pi/2 with the oracle's own ball evaluators
    (independent formulas: asin through atan(x / sqrt(1 - x^2)), acos through
    2 atan(sqrt((1 - x)/(1 + x)))), and arctangent relations against pi."""
    from oracle.functions import _ball_asin, _ball_acos, _ball_atan
    from oracle.consts import pi
    rng = random.Random(13)
    for _ in range(200):
        x = rng.uniform(-1, 1) if rng.random() < 0.5 else \
            math.copysign(1 - 10 ** rng.uniform(-15, 0), rng.random() - 0.5)
        if abs(x) >= 1 or x == 0:
            continue
        s = B.add(_ball_asin(x, 120), _ball_acos(x, 120), 200)
        assert _contains_one(B.div(s, B.scale2(pi(220), -1), 200)), x
    # Euler's and Machin's arctangent relations pin atan against pi, which
    # the oracle computes from its own series (and which is pinned to the
    # AGM): atan 1 = pi/4, atan 1/2 + atan 1/3 = pi/4,
    # 4 atan 1/5 - atan 1/239 = pi/4, 2 atan 1/2 + atan 3/4 = pi/2
    from oracle.elementary import atan_ball
    q = lambda a, b: B.div(B.exact(a), B.exact(b), 260)
    quarter = B.scale2(pi(260), -2)
    checks = [(_ball_atan(1.0, 200), quarter),
              (B.add(atan_ball(q(1, 2), 200), atan_ball(q(1, 3), 200), 240), quarter),
              (B.sub(B.scale2(atan_ball(q(1, 5), 200), 2), atan_ball(q(1, 239), 200), 240),
               quarter),
              (B.add(B.scale2(atan_ball(q(1, 2), 200), 1), atan_ball(q(3, 4), 200), 240),
               B.scale2(quarter, 1))]
    for lhs, rhs in checks:
        assert _contains_one(B.div(lhs, rhs, 240))


def test_asin_acos_atan_small_arguments():
    """asin x, atan x -> x and acos x -> pi/2 - x for tiny x (Taylor)."""
    for x in (1e-300, -3e-200, 5e-324, 2.0 ** -30):
        assert evaluate1("asin", "f64", x)[0] == x
        assert evaluate1("atan", "f64", x)[0] == x
    assert evaluate1("acos", "f64", 5e-324)[0] == evaluate1("acos", "f64", 0.0)[0]
    assert evaluate1("asin", "f64", 2.0 ** -26)[0] == 2.0 ** -26    # x^3/6 < ulp/2
    with mpmath.workprec(400):
        for x in (2.0 ** -20, 0.3, 0.5, 0.9999):
            assert evaluate1("asin", "f64", x)[0] == float(mpmath.asin(mpmath.mpf(x)))


def test_identities_on_balls():
    rng = random.Random(12)
    for _ in range(200):
        x = _rand_bits(rng)
        if not math.isfinite(x) or x == 0:
            continue
        n, d = x.as_integer_ratio()
        k, r = sincos_reduced(n, -(d.bit_length() - 1), 120)
        s, c = sin_cos_ball(r, 120)
        one = B.add(B.mul(s, s, 200), B.mul(c, c, 200), 200)
        assert _contains_one(one)
    for _ in range(200):
        x = rng.uniform(-0.99, 0.99)
        s, c = sinh_cosh_small(B.from_float(x), 120)
        one = B.sub(B.mul(c, c, 200), B.mul(s, s, 200), 200)
        assert _contains_one(one)
    for _ in range(200):
        x = abs(_rand_bits(rng))
        if not math.isfinite(x) or x == 0:
            continue
        n, d = x.as_integer_ratio()
        L = log_ball(n, -(d.bit_length() - 1), 200)
        back = exp_ball(L, 200)
        ratio = B.div(back, B.from_float(x), 200)
        assert _contains_one(ratio)


def test_regression_inputs_are_valid_and_oracle_agrees_with_mpmath():
    """tests/golden/regressions.txt: every value is exactly representable in
    its dtype, and the oracle's binary64 result agrees with mpmath."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "regressions.txt")
    conv = {"f64": np.float64, "f32": np.float32, "f16": np.float16}
    n = 0
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        fn, v, dt, *vals = line.split()
        xs = [float.fromhex(x) for x in vals]
        for x in xs:
            assert float(conv[dt](x)) == x or math.isnan(x), (line, x)
        got = evaluate1(fn, "f64", *xs)[0]
        v = _mp_f64(fn, *xs)
        if v == 0 and len(xs) == 1:
            # mpmath has no signed zero: the host libm gives the Annex F sign
            assert same(got, float(NP_UNARY[fn](np.float64(xs[0])))), (line, got)
        elif v == 0 or not mpmath.isfinite(v):
            assert same(got, _to_f64(v)), (line, got, v)
        else:
            # nearest binary64 to the 400-bit value (mpmath's own float()
            # rounds twice for subnormal results)
            with mpmath.workprec(400):
                d = [abs(mpmath.mpf(c) - v) for c in
                     (got, math.nextafter(got, math.inf), math.nextafter(got, -math.inf))]
            assert d[0] <= d[1] and d[0] <= d[2], (line, got)
        n += 1
    assert n >= 10


# --------------------------------------------------------------------------
# log10, exp10, expm1, log1p, cbrt, hypot
# --------------------------------------------------------------------------

def test_log10_exp10_cbrt_exact_points():
    """log10(10^n) = n, exp10(n) = RN(10^n) (Python's int -> float conversion
    rounds half to even, an independent rounding of the exact integer;
    10^23 is a midpoint), cbrt of exact cubes."""
    for n in range(0, 23):
        assert evaluate1("log10", "f64", float(10 ** n))[0] == float(n)
    for n in range(0, 309):
        assert evaluate1("exp10", "f64", float(n))[0] == float(10 ** n), n
    assert evaluate1("exp10", "f64", 23.0)[0] == 1e23
    assert evaluate1("exp10", "f64", 400.0)[0] == math.inf
    for c in (1, 2, 3, 5, 7, 11, 12345, 2 ** 17 + 1):
        for e in (-40, -3, 0, 3, 30):
            x = math.ldexp(float(c ** 3), 3 * e)
            assert evaluate1("cbrt", "f64", x)[0] == math.ldexp(float(c), e)
            assert evaluate1("cbrt", "f64", -x)[0] == -math.ldexp(float(c), e)
    # binary32: cbrt(27) = 3, log10(1e10) = 10 (1e10 is a binary32 value)
    assert evaluate1("cbrt", "f32", 27.0)[0] == 3.0
    assert evaluate1("log10", "f32", 1e10)[0] == 10.0


def test_expm1_log1p_small_arguments_and_inverse():
    """For |x| < 2^-54, expm1 x and log1p x round to x (x^2/2 is below half an
    ulp); and log1p(expm1(x)) = x within the pair's accuracy (MP identity;
    x > -1, where 1 + expm1 x is not tiny and the identity is well
    conditioned)."""
    for x in (1e-17, -1e-17, 5e-324, -5e-324, 2.0 ** -60, -(2.0 ** -1000)):
        assert evaluate1("expm1", "f64", x)[0] == x
        assert evaluate1("log1p", "f64", x)[0] == x
    rng = random.Random(7)
    for _ in range(60):
        x = 10 ** rng.uniform(-20, 2) if rng.random() < 0.5 else -(10 ** rng.uniform(-20, 0))
        _, h, l = evaluate1("expm1", "f64", x)
        with mpmath.workprec(400):
            y = mpmath.log1p(mpmath.mpf(h) + mpmath.mpf(l))
            assert abs(y - x) <= abs(x) * mpmath.mpf(2) ** -100, x


def test_cbrt_cube_identity():
    rng = random.Random(8)
    for _ in range(80):
        x = _rand_bits(rng)
        if not math.isfinite(x) or x == 0:
            continue
        _, h, l = evaluate1("cbrt", "f64", x)
        with mpmath.workprec(400):
            c = (mpmath.mpf(h) + mpmath.mpf(l)) ** 3
            assert abs(c - x) <= abs(x) * mpmath.mpf(2) ** -100, x


def test_hypot_exact_cases_specials_and_mpmath():
    # Pythagorean triples, scaled; hypot(x, 0) = |x|; symmetric and even
    # (m^2 - n^2, 2mn, m^2 + n^2) with m = 2^26 + 1, n = 2^25 - 1: 52- and 53-bit values
    m, n = 2 ** 26 + 1, 2 ** 25 - 1
    big = (m * m - n * n, 2 * m * n, m * m + n * n)
    for a, b, c in ((3, 4, 5), (5, 12, 13), (20, 21, 29), (119, 120, 169), big):
        if max(a, b, c).bit_length() > 53:
            continue
        for e in (-1070, -20, 0, 40, 900):
            x, y, z = (math.ldexp(float(v), e) for v in (a, b, c))
            if not all(math.isfinite(v) for v in (x, y, z)):
                continue
            for sx in (1, -1):
                assert evaluate1("hypot", "f64", sx * x, y)[0] == z
                assert evaluate1("hypot", "f64", y, sx * x)[0] == z
    for x in (0.0, -0.0, 5e-324, -1.5, 1e308):
        assert same(evaluate1("hypot", "f64", x, 0.0)[0], abs(x))
    for x in (math.inf, -math.inf):
        assert evaluate1("hypot", "f64", x, math.nan)[0] == math.inf
        assert evaluate1("hypot", "f64", math.nan, x)[0] == math.inf
    assert math.isnan(evaluate1("hypot", "f64", math.nan, 1.0)[0])
    assert evaluate1("hypot", "f64", 1.5e308, 1.5e308)[0] == math.inf
    assert evaluate1("hypot", "f64", 1e308, 1e308)[0] == math.hypot(1e308, 1e308)
    rng = random.Random(9)
    for _ in range(150):
        x, y = _rand_bits(rng), _rand_bits(rng)
        if rng.random() < 0.5:
            y = x * 10 ** rng.uniform(-20, 0)
        if not (math.isfinite(x) and math.isfinite(y)):
            continue
        got = evaluate1("hypot", "f64", x, y)[0]
        assert same(got, _to_f64(_mp_f64("hypot", x, y))), (x, y)
        assert same(got, math.hypot(x, y)) or abs(got - math.hypot(x, y)) <= math.ulp(got)


def test_inverse_hyperbolics_identities_and_small_arguments():
    """sinh(asinh x) = x, cosh(acosh x) = x and tanh(atanh x) = x on the
    reference pairs (MP identities); asinh x and atanh x round to x for
    |x| < 2^-27 (x^3/6 and x^3/3 are below half an ulp); acosh near 1
    against sqrt(2d) (1 - d/12 + 3d^2/160), d = x - 1."""
    rng = random.Random(10)
    for _ in range(60):
        x = math.copysign(10 ** rng.uniform(-20, 300), rng.random() - 0.5)
        _, h, l = evaluate1("asinh", "f64", x)
        with mpmath.workprec(400):
            assert abs(mpmath.sinh(mpmath.mpf(h) + mpmath.mpf(l)) - x) <= abs(x) * mpmath.mpf(2) ** -98
        a = 1 + 10 ** rng.uniform(-15, 3)
        _, h, l = evaluate1("acosh", "f64", a)
        with mpmath.workprec(400):
            assert abs(mpmath.cosh(mpmath.mpf(h) + mpmath.mpf(l)) - a) <= a * mpmath.mpf(2) ** -98
        t = math.copysign(10 ** rng.uniform(-20, -0.01), rng.random() - 0.5)
        _, h, l = evaluate1("atanh", "f64", t)
        with mpmath.workprec(400):
            assert abs(mpmath.tanh(mpmath.mpf(h) + mpmath.mpf(l)) - t) <= abs(t) * mpmath.mpf(2) ** -98
    for x in (1e-10, -3e-9, 5e-324, -(2.0 ** -40)):
        assert evaluate1("asinh", "f64", x)[0] == x
        assert evaluate1("atanh", "f64", x)[0] == x
    for k in (30, 40, 50):
        d = 2.0 ** -k
        want = math.sqrt(2 * d) * (1 - d / 12 + 3 * d * d / 160)   # to O(d^3)
        got = evaluate1("acosh", "f64", 1 + d)[0]
        assert abs(got - want) <= 2 * math.ulp(want)


def _erfc_continued_fraction(x, terms=4000):
    """erfc x for x > 0 from Laplace's continued fraction, e^(-x^2)/sqrt(pi) /
    (x + (1/2)/(x + 1/(x + (3/2)/(x + 2/(x + ...))))), evaluated bottom-up
    (a formula independent of the oracle's power series)."""
    x = mpmath.mpf(x)
    t = x
    for k in range(terms, 0, -1):
        t = x + mpmath.mpf(k) / 2 / t
    return mpmath.exp(-x * x) / mpmath.sqrt(mpmath.pi) / t


def test_erf_erfc_identities_series_and_table_values():
    """erf(-x) = -erf x, erfc(-x) = 2 - erfc x and erf x + erfc x = 1 on the
    reference pairs; erfc x for x >= 2 against Laplace's continued fraction;
    erf x against 2x/sqrt(pi) (1 - x^2/3 + x^4/10) for |x| < 2^-20; tabulated
    values erf(1/2), erf(1), erfc(2); erfc of tiny x is 1 and erf of tiny x
    is x (2/sqrt(pi)) rounded."""
    rng = random.Random(12)
    for _ in range(40):
        x = rng.uniform(0.01, 6.5) if rng.random() < 0.7 else 10 ** rng.uniform(-12, 0)
        r1, h1, l1 = evaluate1("erf", "f64", x)
        r2, h2, l2 = evaluate1("erf", "f64", -x)
        assert same(r2, -r1) and h2 == -h1 and l2 == -l1
        c1, ch, cl = evaluate1("erfc", "f64", x)
        c2, dh, dl = evaluate1("erfc", "f64", -x)
        with mpmath.workprec(400):
            s = mpmath.mpf(h1) + mpmath.mpf(l1) + mpmath.mpf(ch) + mpmath.mpf(cl)
            assert abs(s - 1) <= mpmath.mpf(2) ** -100
            t = mpmath.mpf(dh) + mpmath.mpf(dl) + mpmath.mpf(ch) + mpmath.mpf(cl)
            assert abs(t - 2) <= mpmath.mpf(2) ** -100
    for x in [2.0, 2.5, 3.75, 5.0, 8.5, 12.0, 19.25, 26.5, 27.25]:
        _, h, l = evaluate1("erfc", "f64", x)
        with mpmath.workprec(300):
            want = _erfc_continued_fraction(x)
            # the pair's low part is a double: near 2^-1022 it holds no more
            # than 2^-1075 absolute
            tol = want * mpmath.mpf(2) ** -95 + mpmath.mpf(2) ** -1075
            assert abs(mpmath.mpf(h) + mpmath.mpf(l) - want) <= tol, x
    for k in (21, 30, 45, 80, 300):
        x = 1.5 * 2.0 ** -k
        _, h, l = evaluate1("erf", "f64", x)
        with mpmath.workprec(300):
            xm = mpmath.mpf(x)
            want = 2 * xm / mpmath.sqrt(mpmath.pi) * (1 - xm ** 2 / 3 + xm ** 4 / 10)
            # omitted terms below x^6, the pair's own rounding below 2^-104
            assert abs(mpmath.mpf(h) + mpmath.mpf(l) - want) <= want * (xm ** 6 + mpmath.mpf(2) ** -104)
    # Abramowitz and Stegun, Table 7.1, to 20 digits
    assert evaluate1("erf", "f64", 0.5)[0] == float("0.52049987781304653768")
    assert evaluate1("erf", "f64", 1.0)[0] == float("0.84270079294971486934")
    assert evaluate1("erfc", "f64", 2.0)[0] == float("0.0046777349810472658379")
    for x in (5e-324, 1e-300, -1e-20, 2.0 ** -60):
        assert evaluate1("erfc", "f64", x)[0] == 1.0
    assert evaluate1("erf", "f64", 2.0 ** -1000)[0] == 1.1283791670955126 * 2.0 ** -1000


def test_log_series_on_balls_agree_with_exact_log():
    """log_of_ball and log1p_ball (used for the inverse hyperbolics) against
    log_ball on exact dyadics."""
    from oracle.elementary import log_of_ball, log1p_ball
    rng = random.Random(11)
    for _ in range(40):
        m = rng.getrandbits(53) | 1
        e = rng.randint(-1100, 900)
        a = log_ball(m, e, 200)
        b = log_of_ball(B.exact(m, e), 200)
        assert abs(B.approx(a) - B.approx(b)) <= abs(B.approx(a)) * 2.0 ** -150 + 2.0 ** -190
        u_m, u_e = rng.getrandbits(53) | 1, rng.randint(-200, 0)
        c = log1p_ball(B.exact(u_m, u_e), 200)
        # 1 + u = (2^-u_e + u_m) 2^u_e exactly
        d = log_ball((1 << -u_e) + u_m, u_e, 200)
        assert abs(B.approx(c) - B.approx(d)) <= abs(B.approx(d)) * 2.0 ** -150


def test_fdim_fmax_fmin_against_ieee_operations():
    """fdim against the host's IEEE subtraction (binary64 and binary32),
    fmax/fmin against numpy's NaN-ignoring fmax/fmin, and the signed-zero
    order (-0 below +0) on all zero pairs."""
    rng = random.Random(13)
    vals = [0.0, -0.0, math.inf, -math.inf, math.nan, 1.0, -1.0, 5e-324, 1e308, -1e308]
    vals += [_rand_bits(rng) for _ in range(300)] + [rng.uniform(-10, 10) for _ in range(100)]
    vals = [v for v in vals]
    pairs = [(a, b) for a in vals[:60] for b in vals[:60]] + \
        [(rng.choice(vals), rng.choice(vals)) for _ in range(2000)]
    for a, b in pairs:
        got = evaluate1("fdim", "f64", a, b)[0]
        want = math.nan if (math.isnan(a) or math.isnan(b)) else (a - b if a > b else 0.0)
        assert same(got, want), ("fdim", a, b, got, want)
        fa, fb = np.float32(a), np.float32(b)
        got32 = evaluate1("fdim", "f32", float(fa), float(fb))[0]
        with np.errstate(all="ignore"):
            w32 = np.float32("nan") if (np.isnan(fa) or np.isnan(fb)) else \
                (fa - fb if fa > fb else np.float32(0.0))
        assert same(got32, float(w32)), ("fdim f32", fa, fb, got32, w32)
        if a == 0.0 and b == 0.0:
            neg_a, neg_b = math.copysign(1, a) < 0, math.copysign(1, b) < 0
            assert same(evaluate1("fmax", "f64", a, b)[0], -0.0 if (neg_a and neg_b) else 0.0)
            assert same(evaluate1("fmin", "f64", a, b)[0], 0.0 if not (neg_a or neg_b) else -0.0)
            continue
        assert same(evaluate1("fmax", "f64", a, b)[0], float(np.fmax(a, b))), ("fmax", a, b)
        assert same(evaluate1("fmin", "f64", a, b)[0], float(np.fmin(a, b))), ("fmin", a, b)


def test_exact_c99_set_against_host_operations():
    """sqrt against the host's IEEE square root (binary64, and numpy's
    binary32 one), trunc/floor/ceil/rint/fabs/copysign/nextafter against
    numpy, round against decimal's ROUND_HALF_UP on the exact decimal
    expansion, logb against frexp; signs of zero included."""
    import decimal
    rng = random.Random(14)
    xs = [0.0, -0.0, math.inf, -math.inf, 0.5, -0.5, 1.5, -2.5, 2.5, 0.49999999999999994,
          -0.49999999999999994, 4503599627370495.5, 4503599627370497.0, 5e-324, -1e-310,
          1.7976931348623157e308, 4.0, 9.0, 2.0]
    xs += [_rand_bits(rng) for _ in range(400)] + [rng.uniform(-100, 100) for _ in range(200)]
    xs = [x for x in xs if not math.isnan(x)]
    for x in xs:
        want = {"trunc": float(np.trunc(x)), "floor": float(np.floor(x)),
                "ceil": float(np.ceil(x)), "rint": float(np.rint(x)), "fabs": float(np.fabs(x))}
        with np.errstate(invalid="ignore"):
            want["sqrt"] = float(np.sqrt(x))
        if math.isfinite(x):
            d = decimal.Decimal(x).quantize(decimal.Decimal(1), rounding=decimal.ROUND_HALF_UP,
                                            context=decimal.Context(prec=400))
            want["round"] = math.copysign(float(d), x)
            want["logb"] = -math.inf if x == 0 else float(math.frexp(x)[1] - 1)
        else:
            want["round"] = x
            want["logb"] = math.inf
        for fn, w in want.items():
            assert same(evaluate1(fn, "f64", x)[0], w), (fn, x, evaluate1(fn, "f64", x)[0], w)
        f = float(np.float32(x)) if abs(x) < 3e38 or not math.isfinite(x) else 1.0
        with np.errstate(invalid="ignore"):
            w32 = float(np.sqrt(np.float32(f)))
        assert same(evaluate1("sqrt", "f32", f)[0], w32), ("sqrt f32", f)
        y = rng.choice(xs)
        assert same(evaluate1("copysign", "f64", x, y)[0], float(np.copysign(x, y)))
        assert same(evaluate1("nextafter", "f64", x, y)[0], float(np.nextafter(x, y))), (x, y)
        g = float(np.float32(y)) if abs(y) < 3e38 or not math.isfinite(y) else -1.0
        assert same(evaluate1("nextafter", "f32", f, g)[0],
                    float(np.nextafter(np.float32(f), np.float32(g)))), (f, g)


def test_ldexp_ilogb_frexp_against_numpy():
    """The integer-operand functions against numpy's ldexp and frexp (host
    C library), binary64 and binary32, over random patterns, subnormals,
    zeros, infinities and exponents across the whole range."""
    from oracle import intfuncs as I
    rng = random.Random(15)
    xs = [0.0, -0.0, math.inf, -math.inf, 5e-324, -5e-324, 1.0, 0.75, 1.7976931348623157e308]
    xs += [_rand_bits(rng) for _ in range(500)]
    for x in xs:
        if math.isnan(x):
            assert I.ilogb(x) == I.INT_MIN and math.isnan(I.frexp(x)[0])
            continue
        m, e = np.frexp(x)
        assert I.frexp(x) == (float(m), int(e) if math.isfinite(x) else 0) or \
            (not math.isfinite(x) and I.frexp(x)[0] == x)
        want = I.INT_MIN if x == 0 else (I.INT_MAX if math.isinf(x) else int(np.frexp(x)[1]) - 1)
        assert I.ilogb(x) == want, x
        for n in (rng.randint(-2200, 2200), rng.randint(-60, 60), -1074, 1023, 2100):
            assert same(I.ldexp(x, n, "f64"), float(np.ldexp(x, n))), (x, n)
            f = np.float32(x) if abs(x) < 3e38 or not math.isfinite(x) else np.float32(1.5)
            n32 = max(-400, min(400, n))
            with np.errstate(over="ignore", under="ignore"):
                w = float(np.ldexp(f, n32))
            assert same(I.ldexp(float(f), n32, "f32"), w), (float(f), n32)


def test_modf_fma_lrint_lround_against_host():
    """modf against Python's math.modf, fma against the host C library's
    fma, lrint against numpy's rint, lround against decimal's half-up
    rounding (binary64)."""
    import ctypes
    import decimal
    from oracle import intfuncs as I
    libm = ctypes.CDLL("libm.so.6")
    libm.fma.restype = ctypes.c_double
    libm.fma.argtypes = [ctypes.c_double] * 3
    rng = random.Random(16)
    vals = [0.0, -0.0, math.inf, -math.inf, 0.5, -0.5, 2.5, -2.5, 1e19, -1e19, 5e-324]
    vals += [_rand_bits(rng) for _ in range(300)] + [rng.uniform(-1e3, 1e3) for _ in range(200)]
    vals = [v for v in vals if not math.isnan(v)]
    for x in vals:
        f, ip = I.modf(x)
        wf, wip = math.modf(x)
        assert same(f, wf) and same(ip, wip), x
        if math.isfinite(x) and abs(x) < 9.2e18:
            assert I.lrint(x) == int(np.rint(x)), x
            d = decimal.Decimal(x).quantize(decimal.Decimal(1), rounding=decimal.ROUND_HALF_UP,
                                            context=decimal.Context(prec=400))
            assert I.lround(x) == int(d), x
        else:
            assert I.lrint(x) == I.INT64_MIN and I.lround(x) == I.INT64_MIN
    for _ in range(3000):
        a, b, c = (rng.choice(vals) for _ in range(3))
        assert same(I.fma(a, b, c, "f64"), libm.fma(a, b, c)), (a, b, c)


def test_remquo_against_host_libm():
    """remquo against the host C library's remquo (binary64): the remainder
    bit for bit and the quotient's sign and low three bits."""
    import ctypes
    from oracle import intfuncs as I
    libm = ctypes.CDLL("libm.so.6")
    libm.remquo.restype = ctypes.c_double
    libm.remquo.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
    rng = random.Random(17)
    vals = [0.0, -0.0, math.inf, -math.inf, 1.0, -1.0, 0.75, 3.0, 2.5, 5e-324, 1e308]
    vals += [_rand_bits(rng) for _ in range(300)] + [rng.uniform(-50, 50) for _ in range(200)]
    vals = [v for v in vals if not math.isnan(v)]
    for _ in range(4000):
        x, y = rng.choice(vals), rng.choice(vals)
        q = ctypes.c_int(0)
        w = libm.remquo(x, y, ctypes.byref(q))
        r, qq = I.remquo(x, y)
        assert same(r, w), (x, y, r, w)
        if math.isfinite(w) and math.isfinite(y):
            assert qq % 8 == q.value % 8 and (qq == 0 or (qq < 0) == (q.value < 0)), (x, y, qq, q.value)
