"""Rigorous midpoint-radius ("ball") arithmetic on Python integers.

Test infrastructure only: nothing in the library path may import this module.

A Ball ``(m, r, e)`` stands for every real in ``[(m - r) * 2**e, (m + r) * 2**e]``
with integers ``m`` and ``r >= 0``.  Every operation returns a ball that is
guaranteed to contain the exact result of the operation applied to any points
of the argument balls; the midpoint is trimmed to ``prec`` significant bits and
the trimming error is added to the radius.  This is what lets the oracle decide
correct rounding (Ziv's strategy): if both ends of a ball round to the same
floating-point number, that number is the correctly rounded result.

The paper's own tester compares against a multiprecision library (Section 6,
"Testing"); that library is not available here, so the oracle carries its own
arithmetic.  It deliberately shares nothing with the GPU code.
"""
from math import isqrt, ldexp

__all__ = ["Ball", "exact", "from_float", "add", "sub", "mul", "div", "sqrt",
           "neg", "scale2", "contains_zero", "is_positive", "is_negative",
           "approx", "mag_log2", "PrecisionError"]


class PrecisionError(ArithmeticError):
    """Raised when a ball is too wide for an operation (e.g. a divisor ball
    contains zero).  Callers respond by retrying at a higher precision."""


class Ball:
    __slots__ = ("m", "r", "e")

    def __init__(self, m, r, e):
        self.m = m
        self.r = r
        self.e = e

    def __repr__(self):
        return "Ball(%d, %d, %d)" % (self.m, self.r, self.e)

    def lo_hi(self):
        """Exact endpoints as (lo_int, hi_int, e)."""
        return self.m - self.r, self.m + self.r, self.e


def exact(m, e=0):
    return Ball(m, 0, e)


def from_float(x):
    """Exact ball of a finite Python float (binary64; binary32/16 values are
    exactly representable as binary64 as well)."""
    n, d = x.as_integer_ratio()
    return Ball(n, 0, -(d.bit_length() - 1))


def _trim(m, r, e, prec):
    n = abs(m).bit_length()
    if n > prec:
        s = n - prec
        m >>= s                      # floor: |m0 - (m << s)| < 2**s
        r = -((-r) >> s) + 1         # ceil(r / 2**s) + 1 (truncation error)
        e += s
    elif m == 0 and r.bit_length() > prec:
        s = r.bit_length() - prec
        r = -((-r) >> s) + 1
        e += s
    return Ball(m, r, e)


def neg(a):
    return Ball(-a.m, a.r, a.e)


def scale2(a, k):
    """a * 2**k, exact."""
    return Ball(a.m, a.r, a.e + k)


def add(a, b, prec):
    if a.e >= b.e:
        d = a.e - b.e
        return _trim((a.m << d) + b.m, (a.r << d) + b.r, b.e, prec)
    d = b.e - a.e
    return _trim(a.m + (b.m << d), a.r + (b.r << d), a.e, prec)


def sub(a, b, prec):
    return add(a, neg(b), prec)


def mul(a, b, prec):
    am, bm = abs(a.m), abs(b.m)
    r = am * b.r + bm * a.r + a.r * b.r
    return _trim(a.m * b.m, r, a.e + b.e, prec)


def div(a, b, prec):
    """a / b; raises PrecisionError if the divisor ball contains zero."""
    A, B = a.m, b.m
    aA, aB = abs(A), abs(B)
    if aB <= b.r:
        raise PrecisionError("divisor ball contains zero")
    s = prec + aB.bit_length() - aA.bit_length() + 4
    if s < 0:
        s = 0
    q = (aA << s) // aB                 # truncation error < 1
    if (A < 0) != (B < 0):
        q = -q
    num = (a.r * aB + b.r * aA) << s
    den = aB * (aB - b.r)
    rad = -((-num) // den) + 1
    return _trim(q, rad, a.e - b.e - s, prec)


def sqrt(a, prec):
    lo, hi, e = a.lo_hi()
    if lo < 0:
        if hi < 0:
            raise ValueError("sqrt of a negative ball")
        raise PrecisionError("sqrt of a ball containing negative values")
    if e & 1:
        lo <<= 1
        hi <<= 1
        e -= 1
    k = (2 * prec + 6 - hi.bit_length()) // 2
    if k < 0:
        k = 0
    slo = isqrt(lo << (2 * k))          # <= sqrt(lo) * 2**k
    shi = isqrt(hi << (2 * k)) + 1      # >= sqrt(hi) * 2**k
    return _trim(slo + shi, shi - slo, e // 2 - k - 1, prec)


def contains_zero(a):
    return abs(a.m) <= a.r


def is_positive(a):
    return a.m - a.r > 0


def is_negative(a):
    return a.m + a.r < 0


def mag_log2(a):
    """An integer L with |x| < 2**L for every x in the ball."""
    return (abs(a.m) + a.r).bit_length() + a.e


def approx(a):
    """Midpoint as a Python float (may overflow to +-inf or underflow to 0);
    used only for choosing reduction integers, never for results."""
    m, e = a.m, a.e
    n = abs(m).bit_length()
    if n > 60:
        m >>= (n - 60)
        e += (n - 60)
    if e < -1200:
        return 0.0
    try:
        return ldexp(float(m), e)
    except OverflowError:
        return float("inf") if m > 0 else float("-inf")
