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

__all__ = ["ldexp", "ilogb", "frexp", "INT_MIN", "INT_MAX"]

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
