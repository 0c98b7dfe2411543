"""Test infrastructure, not part of the product path: the oracle's C99
functions with integer operands or results -- ldexp(x, n) (scalbn),
ilogb(x), frexp(x) -- written from C99 7.12.6 and F.9.3 (the paper's
library covers all C99 real functions, Section 1).  Only tests/, the smoke
entry and the benchmark's CPU baseline may use this package.

ldexp is x * 2^n rounded once (exact unless it overflows or lands in the
subnormal range); ilogb is the unbiased exponent of x as if normalized, with
FP_ILOGB0 = FP_ILOGBNAN = INT_MIN and INT_MAX for infinities (the values of
the common x86-64 C library); frexp splits x into m * 2^e with |m| in
[0.5, 1), zero, infinity and NaN giving (x, 0)."""
import math

from .functions import _dyadic
from .rounding import FORMATS, rn_dyadic

__all__ = ["ldexp", "ilogb", "frexp", "modf", "fma", "lrint", "lround", "remquo", "INT_MIN", "INT_MAX",
           "INT64_MIN"]

INT_MIN = -2 ** 31
INT_MAX = 2 ** 31 - 1


def ldexp(x, n, fmt_name):
    """x * 2**n rounded to nearest-even in the format (x a value of it)."""
    if math.isnan(x) or math.isinf(x) or x == 0.0:
        return x
    m, e = _dyadic(abs(x))
    v = rn_dyadic(m, e + int(n), FORMATS[fmt_name])
    return math.copysign(v, x)


def ilogb(x):
    if math.isnan(x) or x == 0.0:
        return INT_MIN
    if math.isinf(x):
        return INT_MAX
    m, e = _dyadic(abs(x))
    return e + m.bit_length() - 1


def frexp(x):
    """(m, e) with x = m * 2**e and 0.5 <= |m| < 1 (exact)."""
    if math.isnan(x) or math.isinf(x) or x == 0.0:
        return x, 0
    e = ilogb(x) + 1
    return math.ldexp(x, -e), e


# ---------------------------------------------------------------------------
# modf, fma, lrint, lround (C99 7.12.6.12, 7.12.13.1, 7.12.9.5, 7.12.9.7)
# ---------------------------------------------------------------------------
INT64_MIN = -2 ** 63


def modf(x):
    """(fractional part, integral part), both with the sign of x; inf gives
    (+-0, +-inf), NaN (NaN, NaN)."""
    if math.isnan(x):
        return x, x
    if math.isinf(x):
        return math.copysign(0.0, x), x
    ip = float(math.trunc(x))
    return math.copysign(x - ip, x), math.copysign(ip, x)


def fma(x, y, z, fmt_name):
    """x * y + z rounded once (IEEE fusedMultiplyAdd), with the invalid
    cases (inf * 0, inf - inf) NaN and an exact zero signed by the rules of
    IEEE addition."""
    from fractions import Fraction
    if math.isnan(x) or math.isnan(y) or math.isnan(z):
        return math.nan
    if (math.isinf(x) and y == 0.0) or (math.isinf(y) and x == 0.0):
        return math.nan
    if math.isinf(x) or math.isinf(y):
        p = math.copysign(math.inf, x) * math.copysign(1.0, y)
        if math.isinf(z) and z != p:
            return math.nan
        return p
    if math.isinf(z):
        return z
    v = Fraction(x) * Fraction(y) + Fraction(z)
    if v == 0:
        pneg = (math.copysign(1.0, x) < 0) != (math.copysign(1.0, y) < 0)
        pzero = x == 0.0 or y == 0.0
        if pzero and z == 0.0:
            return -0.0 if (pneg and math.copysign(1.0, z) < 0) else 0.0
        return 0.0
    num, den = v.numerator, v.denominator
    # den is a power of two
    return rn_dyadic(num, -(den.bit_length() - 1), FORMATS[fmt_name])


def lrint(x):
    """The nearest integer (ties to even) as int64; INT64_MIN where it does
    not fit (and for NaN), as the x86-64 conversion gives."""
    from fractions import Fraction
    if math.isnan(x) or math.isinf(x):
        return INT64_MIN
    k = round(Fraction(x))
    return k if -2 ** 63 <= k < 2 ** 63 else INT64_MIN


def lround(x):
    """The nearest integer (ties away from zero) as int64; INT64_MIN where it
    does not fit (and for NaN)."""
    from fractions import Fraction
    if math.isnan(x) or math.isinf(x):
        return INT64_MIN
    q = Fraction(x)
    k = math.floor(abs(q) + Fraction(1, 2))
    k = -k if q < 0 else k
    return k if -2 ** 63 <= k < 2 ** 63 else INT64_MIN


def remquo(x, y):
    """(remainder(x, y), quo): quo has the sign of x/y and the low three
    bits of the magnitude of the quotient rounded to nearest-even (C99
    7.12.10.3); NaN remainder and quo 0 for y = 0, infinite x or NaN; x and
    quo 0 for infinite y."""
    from fractions import Fraction
    if math.isnan(x) or math.isnan(y) or math.isinf(x) or y == 0.0:
        return math.nan, 0
    if math.isinf(y):
        return x, 0
    q = round(Fraction(x) / Fraction(y))            # ties to even
    r = Fraction(x) - q * Fraction(y)                # exact, representable
    rv = float(r) if r != 0 else math.copysign(0.0, x)
    neg = (math.copysign(1.0, x) < 0) != (math.copysign(1.0, y) < 0)
    mag = abs(q) & 7
    return rv, (-mag if neg else mag)
