"""Binary floating-point formats and round-to-nearest-even of exact dyadics.

Test infrastructure only: nothing in the library path may import this module.

The paper's functions assume round-to-nearest mode only (Section 5, "Handling
of Special Numbers, Exception and Flags"); the oracle's reference value for a
finite input is therefore RN(f(x)) in the output format, with gradual
underflow and overflow to infinity, as IEEE 754 defines it.
"""
import math
from collections import namedtuple

__all__ = ["Format", "FORMATS", "rn_dyadic", "rn_ball", "ulp_exponent"]

# p: precision incl. the hidden bit; emin/emax: exponents of the smallest and
# largest normal binades.
Format = namedtuple("Format", "name p emin emax")

FORMATS = {
    "f64": Format("f64", 53, -1022, 1023),
    "f32": Format("f32", 24, -126, 127),
    "bf16": Format("bf16", 8, -126, 127),
    "f16": Format("f16", 11, -14, 15),
}

INF = float("inf")


def rn_dyadic(m, e, fmt, zero_sign=1):
    """Round the exact value m * 2**e (m, e integers) to nearest-even in fmt.

    Returns a Python float (every value of the four formats is exactly a
    binary64).  ``zero_sign`` gives the sign of a zero input (m == 0)."""
    if m == 0:
        return 0.0 if zero_sign > 0 else -0.0
    neg = m < 0
    a = -m if neg else m
    n = a.bit_length()
    lead = e + n - 1                     # exponent of the leading bit
    if lead > fmt.emax + 1:
        return -INF if neg else INF
    q_e = max(lead, fmt.emin) - (fmt.p - 1)   # weight of the last kept bit
    if q_e <= e:
        q = a << (e - q_e)
    else:
        s = q_e - e
        if s > n + 1:
            q = 0                        # far below half the smallest step
        else:
            q = a >> s
            rem = a - (q << s)
            half = 1 << (s - 1)
            if rem > half or (rem == half and (q & 1)):
                q += 1
    # overflow: the rounded magnitude reached 2**(emax+1)
    if q.bit_length() + q_e - 1 > fmt.emax:
        return -INF if neg else INF
    if q == 0:
        return -0.0 if neg else 0.0
    v = math.ldexp(float(q), q_e)        # exact: q has <= p <= 53 bits
    return -v if neg else v


def rn_ball(b, fmt):
    """Correctly rounded value of every point of the ball, or None when the
    ball's ends round differently (the caller must raise the precision)."""
    lo, hi, e = b.lo_hi()
    if lo <= 0 <= hi and not (lo == 0 and hi == 0):
        return None
    x = rn_dyadic(lo, e, fmt)
    y = rn_dyadic(hi, e, fmt)
    if x == y and math.copysign(1.0, x) == math.copysign(1.0, y):
        return x
    return None


def ulp_exponent(v_abs_log2_floor, fmt):
    """Exponent of ulp(v) for a value whose binade exponent is given."""
    return max(v_abs_log2_floor, fmt.emin) - (fmt.p - 1)
