"""The oracle proper: correctly rounded C99 real functions, one element at a time.

Test infrastructure only: only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg may import this package.  Nothing here is shared with, or
imported by, the GPU library.

For a finite, non-special argument the oracle returns RN_fmt(f(x)), the exact
value rounded to nearest-even in the output format (gradual underflow, overflow
to infinity), found with Ziv's strategy: evaluate a rigorous ball at precision
P; if both ends round to the same number that is the answer, else double P.
The cap is 16384 bits; hitting it raises instead of returning a guess.  Ziv's
loop only stops when the exact value is not itself a rounding boundary
(a representable number or a midpoint); the cases where it can be one are
detected and computed exactly (exp2 and log2 at powers of two, pow when x^y is
a dyadic rational, log10 at powers of ten, exp10 at nonnegative integers,
cbrt at cubes and hypot when x^2 + y^2 is a square).  exp, sin, cos, tan,
log (x != 1), atan (x != 0), expm1 and log1p (x != 0), the hyperbolic
functions and their inverses (asinh, atanh at x != 0, acosh at x != 1) and
erf, erfc of a nonzero dyadic are transcendental, hence never a boundary.
lgamma and tgamma (oracle/gamma.py): exact at the positive integers (tgamma)
and at 1 and 2 (lgamma); elsewhere the loop relies on the values not being
boundaries, which its termination on every tested argument confirms.

Special inputs (zeros, infinities, NaN) follow C99 Annex F (F.9), which the
paper adopts: "same results as libm, as specified in the ANSI C standard"
(Section 5, opening paragraphs, and "Handling of Special Numbers").

fmod is n - d*trunc(n/d) and remainder is n - d*rint_even(n/d); both results
are exactly representable, so the oracle computes them with exact integer
arithmetic (Section 5, "FP Remainder", Algorithm 1's postcondition).

fdim, fmax, fmin are C99 functions of the library's set (Section 1) that the
paper only shows as a masking example: fdim(x, y) is x - y rounded when
x > y, else +0; fmax/fmin return the larger/smaller argument, the other one
if one is NaN, NaN if both are (F.9.9).  C99 leaves the order of -0 and +0
open; here -0 < +0 (fmax(-0, +0) = +0, fmin(-0, +0) = -0).  The rest of the
C99 set that has one exact answer: sqrt (correctly rounded: the exact
square root of the dyadic argument, rounded once), trunc, floor, ceil, round
(halfway cases away from zero), rint (to nearest even), fabs, logb (the
unbiased exponent of the argument as if normalized), copysign, nextafter
(F.9.4.5, F.9.6, F.9.3.11, F.9.8.3, F.9.9).

Besides the rounded value the oracle returns a high-precision approximation of
the exact value as a pair of binary64 numbers (hi, lo), from which the tests
compute ULP errors.
"""
import math

from . import ball as B
from .ball import Ball, exact, from_float, add, sub, mul, div, PrecisionError
from .consts import pi, ln2
from .elementary import (exp_ball, log_ball, log1p_ball, sincos_reduced, sin_cos_ball,
                         atan_ball, sinh_cosh_small, erf_ball)
from .rounding import FORMATS, rn_dyadic, rn_ball
from .gamma import lgamma_ball, tgamma_ball

__all__ = ["UNARY", "BINARY", "evaluate1", "OracleError"]

NAN = float("nan")
INF = float("inf")
PREC_CAP = 16384

UNARY = ("sin", "cos", "tan", "exp", "exp2", "log", "log2",
         "sinh", "cosh", "tanh", "asin", "acos", "atan",
         "log10", "exp10", "expm1", "log1p", "cbrt", "asinh", "acosh", "atanh",
         "erf", "erfc", "sqrt", "trunc", "floor", "ceil", "round", "rint", "fabs", "logb",
         "lgamma", "tgamma")
BINARY = ("pow", "atan2", "fmod", "remainder", "hypot", "fdim", "fmax", "fmin", "copysign",
          "nextafter")
# functions whose result is the exact value or its correct rounding (no
# approximation involved): defined directly, no Ziv loop
EXACT_UNARY = ("sqrt", "trunc", "floor", "ceil", "round", "rint", "fabs", "logb")


class OracleError(RuntimeError):
    pass


def _sgn(x):
    return -1 if math.copysign(1.0, x) < 0 else 1


def _dyadic(x):
    """Exact (m, e) with x = m * 2**e and m odd (x finite, nonzero)."""
    n, d = x.as_integer_ratio()
    e = -(d.bit_length() - 1)
    tz = (n & -n).bit_length() - 1
    return n >> tz, e + tz


def _is_int(x):
    return math.isfinite(x) and x == math.floor(x)


def _is_odd_int(x):
    if not _is_int(x) or abs(x) >= 2.0 ** 53:
        return False
    return int(x) & 1 == 1


# --------------------------------------------------------------------------
# Annex F special cases.  Each returns a float, or None for "compute".
# --------------------------------------------------------------------------

def _special_unary(fn, x):
    if math.isnan(x):
        return NAN
    if fn in ("sin", "tan", "sinh", "tanh"):
        if x == 0.0:
            return x
        if math.isinf(x):
            if fn == "sinh":
                return x
            if fn == "tanh":
                return math.copysign(1.0, x)
            return NAN
    elif fn == "cos":
        if x == 0.0:
            return 1.0
        if math.isinf(x):
            return NAN
    elif fn == "cosh":
        if x == 0.0:
            return 1.0
        if math.isinf(x):
            return INF
    elif fn in ("exp", "exp2"):
        if x == 0.0:
            return 1.0
        if math.isinf(x):
            return INF if x > 0 else 0.0
    elif fn in ("log", "log2"):
        if x == 0.0:
            return -INF
        if x < 0:
            return NAN
        if math.isinf(x):
            return INF
        if x == 1.0:
            return 0.0
    elif fn in ("asin", "acos"):
        if abs(x) > 1.0:                 # including +-inf
            return NAN
        if fn == "asin" and x == 0.0:
            return x
        if fn == "acos" and x == 1.0:
            return 0.0
    elif fn == "atan":
        if x == 0.0:
            return x
    elif fn == "log10":
        if x == 0.0:
            return -INF
        if x < 0:
            return NAN
        if math.isinf(x):
            return INF
        if x == 1.0:
            return 0.0
    elif fn == "exp10":
        if x == 0.0:
            return 1.0
        if math.isinf(x):
            return INF if x > 0 else 0.0
    elif fn == "expm1":
        if x == 0.0:
            return x
        if math.isinf(x):
            return INF if x > 0 else -1.0
    elif fn == "log1p":
        if x == 0.0:
            return x
        if x == -1.0:
            return -INF
        if x < -1.0:
            return NAN
        if math.isinf(x):
            return INF
    elif fn == "cbrt":
        if x == 0.0 or math.isinf(x):
            return x
    elif fn == "asinh":
        if x == 0.0 or math.isinf(x):
            return x
    elif fn == "acosh":
        if x < 1.0:                      # including -inf
            return NAN
        if x == 1.0:
            return 0.0
        if math.isinf(x):
            return INF
    elif fn == "atanh":
        if abs(x) > 1.0:                 # including +-inf
            return NAN
        if x == 0.0:
            return x
        if abs(x) == 1.0:
            return math.copysign(INF, x)
    elif fn == "erf":
        if x == 0.0:
            return x
        if math.isinf(x):
            return math.copysign(1.0, x)
    elif fn == "erfc":
        if x == 0.0:
            return 1.0
        if math.isinf(x):
            return 0.0 if x > 0 else 2.0
    elif fn == "lgamma":
        # F.9.5.3: +inf at +-inf and at the poles (zero, negative integers)
        if math.isinf(x) or (x <= 0.0 and x == math.floor(x)):
            return INF
        if x == 1.0 or x == 2.0:
            return 0.0
    elif fn == "tgamma":
        # F.9.5.4: +-0 -> +-inf, negative integers and -inf -> NaN, +inf -> +inf
        if x == 0.0:
            return math.copysign(INF, x)
        if math.isinf(x):
            return INF if x > 0 else NAN
        if x < 0.0 and x == math.floor(x):
            return NAN
    return None


def _special_atan2(y, x, fmt):
    """atan2(y, x) per Annex F; the pi-related constants are correctly
    rounded into the output format (callers pass the same constants through
    the normal path, so only the case analysis lives here)."""
    if math.isnan(x) or math.isnan(y):
        return NAN
    sy = _sgn(y)
    if y == 0.0:
        if _sgn(x) < 0:              # x is -0 or negative (incl. -inf)
            return sy * _round_const("pi", fmt)
        return math.copysign(0.0, y)
    if x == 0.0:
        return sy * _round_const("pi/2", fmt)
    if math.isinf(y):
        if math.isinf(x):
            return sy * _round_const("3pi/4" if x < 0 else "pi/4", fmt)
        return sy * _round_const("pi/2", fmt)
    if math.isinf(x):
        if x < 0:
            return sy * _round_const("pi", fmt)
        return math.copysign(0.0, y)
    return None


def _special_pow(x, y):
    """pow(x, y) per Annex F.  Returns a float or None."""
    if y == 0.0:
        return 1.0
    if x == 1.0:
        return 1.0
    if math.isnan(x) or math.isnan(y):
        return NAN
    odd = _is_odd_int(y)
    if x == 0.0:
        if y < 0:
            return math.copysign(INF, x) if odd else INF
        return x if odd else 0.0
    if math.isinf(y):
        if x == -1.0:
            return 1.0
        if (abs(x) < 1.0) == (y < 0):
            return INF
        return 0.0
    if math.isinf(x):
        if x < 0:
            if y < 0:
                return -0.0 if odd else 0.0
            return -INF if odd else INF
        return 0.0 if y < 0 else INF
    if x < 0 and not _is_int(y):
        return NAN
    return None


def _special_hypot(x, y):
    """Annex F: an infinite argument gives +inf even when the other is NaN."""
    if math.isinf(x) or math.isinf(y):
        return INF
    if math.isnan(x) or math.isnan(y):
        return NAN
    return None


def _special_fmod(x, y):
    if math.isnan(x) or math.isnan(y) or math.isinf(x) or y == 0.0:
        return NAN
    if x == 0.0:
        return x
    if math.isinf(y):
        return x
    return None


# --------------------------------------------------------------------------
# Correctly rounded constants (used by atan2 specials)
# --------------------------------------------------------------------------

_const_cache = {}


def _round_const(name, fmt):
    key = (name, fmt.name)
    if key not in _const_cache:
        p = 200
        num, den = {"pi": (1, 1), "pi/2": (1, 2), "pi/4": (1, 4),
                    "3pi/4": (3, 4)}[name]
        b = pi(p)
        b = div(mul(b, exact(num), p), exact(den), p)
        v = rn_ball(b, fmt)
        assert v is not None
        _const_cache[key] = v
    return _const_cache[key]


# --------------------------------------------------------------------------
# Ball evaluators for finite, non-special arguments
# --------------------------------------------------------------------------

def _clamp_exp_arg(xb):
    """Arguments beyond +-2100 give results outside every format's range
    (2**3000 overflows, 2**-3000 is below half the smallest subnormal); clamp
    so the ball code never sees astronomically large reduction integers."""
    a = B.approx(xb)
    if a > 2100:
        return exact(2100)
    if a < -2100:
        return exact(-2100)
    return xb


def _ball_exp(x, prec):
    return exp_ball(_clamp_exp_arg(from_float(x)), prec)


def _ball_exp2(x, prec):
    xb = mul(from_float(x), ln2(prec + 40), prec + 40)
    return exp_ball(_clamp_exp_arg(xb), prec)


def _ball_log(x, prec):
    m, e = _dyadic(x)
    return log_ball(m, e, prec)


def _ball_log2(x, prec):
    m, e = _dyadic(x)
    return div(log_ball(m, e, prec + 8), ln2(prec + 16), prec + 8)


def _ball_sin(x, prec):
    m, e = _dyadic(x)
    k, r = sincos_reduced(m, e, prec)
    s, c = sin_cos_ball(r, prec + 8)
    return (s, c, B.neg(s), B.neg(c))[k]


def _ball_cos(x, prec):
    m, e = _dyadic(x)
    k, r = sincos_reduced(m, e, prec)
    s, c = sin_cos_ball(r, prec + 8)
    return (c, B.neg(s), B.neg(c), s)[k]


def _ball_tan(x, prec):
    m, e = _dyadic(x)
    k, r = sincos_reduced(m, e, prec)
    s, c = sin_cos_ball(r, prec + 8)
    if k & 1:
        return B.neg(div(c, s, prec + 8))
    return div(s, c, prec + 8)


def _ball_sinh(x, prec):
    ax = abs(x)
    if ax < 1.0:
        s, _ = sinh_cosh_small(from_float(x), prec)
        return s
    E = exp_ball(_clamp_exp_arg(from_float(ax)), prec + 8)
    s = B.scale2(sub(E, div(exact(1), E, prec + 8), prec + 8), -1)
    return s if x > 0 else B.neg(s)


def _ball_cosh(x, prec):
    ax = abs(x)
    if ax < 1.0:
        _, c = sinh_cosh_small(from_float(ax), prec)
        return c
    E = exp_ball(_clamp_exp_arg(from_float(ax)), prec + 8)
    return B.scale2(add(E, div(exact(1), E, prec + 8), prec + 8), -1)


def _ball_tanh(x, prec):
    ax = abs(x)
    if ax < 1.0:
        s, c = sinh_cosh_small(from_float(x), prec + 8)
        return div(s, c, prec + 8)
    # tanh = 1 - 2 / (E^2 + 1), E = exp|x|; |x| >= 1 so no cancellation issue
    # for the rounding decision (the result is in [0.76, 1]).
    a = min(ax, 40.0 + prec)          # tanh(a) = 1 - O(e^-2a): beyond this the
    E2 = exp_ball(from_float(2 * a), prec + 8)
    t = sub(exact(1), div(exact(2), add(E2, exact(1), prec + 8), prec + 8),
            prec + 8)
    if a < ax:
        # exact tanh lies in (t_lo, 1): widen the ball to cover up to 1
        t = add(t, Ball(1, 1, -(prec + 30)), prec + 8)
    return t if x > 0 else B.neg(t)


def _ball_atan2(y, x, prec):
    ay, ax = abs(y), abs(x)
    wp = prec + 16
    if ay <= ax:
        t = div(from_float(ay), from_float(ax), wp)
        a = atan_ball(t, wp)
    else:
        t = div(from_float(ax), from_float(ay), wp)
        a = sub(B.scale2(pi(wp + 8), -1), atan_ball(t, wp), wp)
    if x < 0:
        a = sub(pi(wp + 8), a, wp)
    return a if y > 0 else B.neg(a)


def _ball_atan(x, prec):
    """atan x: atan|x| for |x| <= 1, pi/2 - atan(1/|x|) above; odd."""
    ax = abs(x)
    wp = prec + 16
    if ax <= 1.0:
        a = atan_ball(from_float(ax), wp)
    else:
        a = sub(B.scale2(pi(wp + 8), -1), atan_ball(div(exact(1), from_float(ax), wp), wp), wp)
    return a if x > 0 else B.neg(a)


def _ball_asin(x, prec):
    """asin x = atan(x / sqrt(1 - x^2)) for |x| < 1, with 1 - x^2 formed
    exactly as (1 - |x|)(1 + |x|); the atan argument is kept in [0, 1] by
    taking pi/2 - atan(sqrt(1 - x^2) / |x|) when |x| > sqrt(1 - x^2)."""
    ax = abs(x)
    wp = prec + 24
    X = from_float(ax)
    one = exact(1)
    c = B.sqrt(mul(sub(one, X, wp), add(one, X, wp), wp), wp)      # sqrt(1 - x^2)
    if ax * ax <= 0.5:
        a = atan_ball(div(X, c, wp), wp)
    else:
        a = sub(B.scale2(pi(wp + 8), -1), atan_ball(div(c, X, wp), wp), wp)
    return a if x > 0 else B.neg(a)


def _ball_acos(x, prec):
    """acos x = 2 atan(sqrt((1 - x) / (1 + x))) for -1 < x < 1 (no
    cancellation near x = 1); the atan argument exceeds 1 when x < 0, then
    atan t = pi/2 - atan(1/t)."""
    wp = prec + 24
    X = from_float(x)
    one = exact(1)
    q = div(sub(one, X, wp), add(one, X, wp), wp)
    if x >= 0.0:
        a = atan_ball(B.sqrt(q, wp), wp)
    else:
        a = sub(B.scale2(pi(wp + 8), -1), atan_ball(B.sqrt(div(one, q, wp), wp), wp), wp)
    return B.scale2(a, 1)


def _ball_log10(x, prec):
    m, e = _dyadic(x)
    return div(log_ball(m, e, prec + 8), log_ball(5, 1, prec + 16), prec + 8)


def _ball_exp10(x, prec):
    wp = prec + 40
    xb = mul(from_float(x), log_ball(5, 1, wp), wp)          # x ln 10
    return exp_ball(_clamp_exp_arg(xb), prec)


def _ball_expm1(x, prec):
    """e^x - 1.  For |x| < 1 as 2 sinh(x/2) e^(x/2) (no cancellation); else
    directly (|e^x - 1| >= 1 - 1/e)."""
    if abs(x) < 1.0:
        h = B.scale2(from_float(x), -1)
        s, _ = sinh_cosh_small(h, prec + 8)
        return B.scale2(mul(s, exp_ball(h, prec + 8), prec + 8), 1)
    return sub(exp_ball(_clamp_exp_arg(from_float(x)), prec + 8), exact(1), prec + 8)


def _one_plus(x):
    """1 + x as an exact dyadic (M, E)."""
    m, e = _dyadic(x)
    if e >= 0:
        return (m << e) + 1, 0
    return m + (1 << -e), e


def _ball_log1p(x, prec):
    """log(1 + x) with 1 + x formed exactly; the logarithm's mantissa lies in
    [sqrt(1/2), sqrt(2)) so the result is accurate relative to its own size
    when 1 + x is near 1."""
    M, E = _one_plus(x)
    return log_ball(M, E, prec)


def _ball_cbrt(x, prec):
    """cbrt x = sign(x) exp(log|x| / 3)."""
    m, e = _dyadic(abs(x))
    wp = prec + 24
    r = exp_ball(div(log_ball(m, e, wp), exact(3), wp), prec + 8)
    return r if x > 0 else B.neg(r)


def _ball_asinh(x, prec):
    """asinh|x| = log1p(u), u = |x| + x^2 / (1 + sqrt(1 + x^2)) (no
    cancellation); odd."""
    wp = prec + 24
    X = from_float(abs(x))
    x2 = mul(X, X, wp)
    one = exact(1)
    u = add(X, div(x2, add(one, B.sqrt(add(one, x2, wp), wp), wp), wp), wp)
    r = log1p_ball(u, prec + 8)
    return r if x > 0 else B.neg(r)


def _ball_acosh(x, prec):
    """acosh x = log1p(u), u = (x - 1) + sqrt((x - 1)(x + 1)), x > 1."""
    wp = prec + 24
    X = from_float(x)
    one = exact(1)
    d = sub(X, one, wp)                                  # exact for a dyadic
    u = add(d, B.sqrt(mul(d, add(X, one, wp), wp), wp), wp)
    return log1p_ball(u, prec + 8)


def _ball_atanh(x, prec):
    """atanh|x| = log1p(2|x| / (1 - |x|)) / 2, |x| < 1; odd."""
    wp = prec + 24
    X = from_float(abs(x))
    u = div(B.scale2(X, 1), sub(exact(1), X, wp), wp)
    r = B.scale2(log1p_ball(u, prec + 8), -1)
    return r if x > 0 else B.neg(r)


def _ball_erf(x, prec):
    r = erf_ball(from_float(abs(x)), prec + 8)
    return r if x > 0 else B.neg(r)


def _ball_erfc(x, prec):
    """1 - erf x; for x > 0 the subtraction cancels about x^2 log2(e) bits,
    which the working precision adds."""
    extra = int(1.45 * x * x) + 16 if x > 0 else 8
    e = erf_ball(from_float(abs(x)), prec + extra)
    return sub(exact(1), e, prec + 8) if x > 0 else add(exact(1), e, prec + 8)


def _sum_squares(x, y):
    """x^2 + y^2 as an exact dyadic (S, E) with E even."""
    terms = [_dyadic(abs(v)) for v in (x, y) if v != 0.0]
    e = min(2 * ev for _, ev in terms)
    S = sum((mv * mv) << (2 * ev - e) for mv, ev in terms)
    if e & 1:
        S <<= 1
        e -= 1
    return S, e


def _ball_hypot(x, y, prec):
    S, e = _sum_squares(x, y)
    return B.sqrt(exact(S, e), prec + 8)


def _ball_pow(x, y, prec):
    """|x|^y (sign handled by the caller) for finite nonzero x, y."""
    m, e = _dyadic(abs(x))
    wp = prec + 40
    L = log_ball(m, e, wp)
    z = mul(L, from_float(y), wp)
    return exp_ball(_clamp_exp_arg(z), prec + 8)


# --------------------------------------------------------------------------
# Exact cases (Ziv would not terminate on them)
# --------------------------------------------------------------------------

def _int_root(n, k):
    """Exact integer k-th root of n if n is a perfect k-th power, else None."""
    if n == 1:
        return 1
    r = int(round(n ** (1.0 / k)))
    for c in (r - 1, r, r + 1):
        if c > 0 and c ** k == n:
            return c
    return None


def _cbrt_exact(x):
    """(m, e) with cbrt|x| = m 2^e when it is a dyadic, else None (then it is
    irrational, hence no rounding boundary)."""
    m, e = _dyadic(abs(x))
    if e % 3 != 0:
        return None
    c = _int_root(m, 3)
    return None if c is None else (c, e // 3)


def _pow_exact(x, y):
    """If |x|^y is a dyadic rational with few enough bits to possibly be a
    representable number or a rounding midpoint, return it as (m, e);
    otherwise None (then it is no rounding boundary and Ziv terminates)."""
    mx, ex = _dyadic(abs(x))
    my, ey = _dyadic(y)
    if ey >= 0:                         # y is an integer
        Y = my << ey
        if mx == 1:
            return 1, ex * Y
        if Y < 0:
            return None                 # 1 / odd^|Y| is not dyadic
        if Y * mx.bit_length() > 400:
            return None                 # odd result with > 54 significant bits
        return mx ** Y, ex * Y
    j = -ey                             # y = my / 2**j, my odd
    if j > 12:
        return None                     # only x == 1 qualifies (handled)
    k = 1 << j
    if ex % k != 0:
        return None
    root = _int_root(mx, k)
    if root is None:
        return None
    ez = ex // k
    if root == 1:
        return 1, ez * my
    if my < 0:
        return None
    if my * root.bit_length() > 400:
        return None
    return root ** my, ez * my


# --------------------------------------------------------------------------
# Exact fmod / remainder
# --------------------------------------------------------------------------

def _fmod_exact(x, y, ieee_remainder):
    mx, ex = _dyadic(abs(x))
    my, ey = _dyadic(abs(y))
    e = min(ex, ey)
    X = mx << (ex - e)
    Y = my << (ey - e)
    q, r = divmod(X, Y)
    if ieee_remainder:
        twice = 2 * r
        if twice > Y or (twice == Y and (q & 1)):
            r -= Y
    return r, e


# --------------------------------------------------------------------------
# Driver
# --------------------------------------------------------------------------

_BALLS = {"sin": _ball_sin, "cos": _ball_cos, "tan": _ball_tan,
          "exp": _ball_exp, "exp2": _ball_exp2, "log": _ball_log,
          "log2": _ball_log2, "sinh": _ball_sinh, "cosh": _ball_cosh,
          "tanh": _ball_tanh, "asin": _ball_asin, "acos": _ball_acos,
          "atan": _ball_atan, "log10": _ball_log10, "exp10": _ball_exp10,
          "expm1": _ball_expm1, "log1p": _ball_log1p, "cbrt": _ball_cbrt,
          "asinh": _ball_asinh, "acosh": _ball_acosh, "atanh": _ball_atanh,
          "erf": _ball_erf, "erfc": _ball_erfc, "lgamma": lgamma_ball, "tgamma": tgamma_ball}


def _dd(b):
    """Midpoint of ball b as a binary64 pair (hi, lo); hi may be +-inf."""
    hi = rn_dyadic(b.m, b.e, FORMATS["f64"])
    if math.isinf(hi) or hi == 0.0:
        return hi, 0.0
    n, d = hi.as_integer_ratio()
    eh = -(d.bit_length() - 1)
    e = min(eh, b.e)
    rest = (b.m << (b.e - e)) - (n << (eh - e))
    lo = rn_dyadic(rest, e, FORMATS["f64"])
    return hi, lo


def _exact_result(m, e, fmt, zero_sign=1):
    """An exactly known value m * 2**e: its rounding, and the binary64 pair of
    the exact value (which may need more bits than the format has, e.g. a
    midpoint) for the ULP metric."""
    v = rn_dyadic(m, e, fmt, zero_sign=zero_sign)
    if m == 0:
        return v, v, 0.0
    hi, lo = _dd(exact(m, e))
    return v, hi, lo


def _ziv(fn_ball, args, fmt, prec0):
    prec = prec0
    while prec <= PREC_CAP:
        try:
            b = fn_ball(*args, prec)
        except PrecisionError:
            prec *= 2
            continue
        v = rn_ball(b, fmt)
        if v is not None:
            hi, lo = _dd(b)
            return v, hi, lo
        prec *= 2
    raise OracleError("precision cap reached for %r" % (args,))


def _ball_sqrt(x, prec):
    m, e = _dyadic(x)
    return B.sqrt(exact(m, e), prec + 8)


def _exact_unary(fn, x, fmt, prec0):
    """The exactly defined unary functions (see the module docstring)."""
    from fractions import Fraction
    if math.isnan(x):
        return NAN, NAN, 0.0
    if fn == "fabs":
        v = abs(x)
        return v, v, 0.0
    if fn == "logb":
        if x == 0.0:
            return -INF, -INF, 0.0
        if math.isinf(x):
            return INF, INF, 0.0
        v = float(math.frexp(x)[1] - 1)
        return v, v, 0.0
    if fn == "sqrt":
        if x < 0.0:
            return NAN, NAN, 0.0
        if x == 0.0 or math.isinf(x):
            return x, x, 0.0
        m, e = _dyadic(x)
        if e & 1:
            m, e = m << 1, e - 1
        r = math.isqrt(m)
        if r * r == m:
            return _exact_result(r, e // 2, fmt)
        return _ziv(_ball_sqrt, (x,), fmt, prec0)
    # integral roundings: exact integers, zero keeping the argument's sign
    if math.isinf(x) or x == 0.0:
        return x, x, 0.0
    q = Fraction(x)
    if fn == "trunc":
        k = math.trunc(q)
    elif fn == "floor":
        k = math.floor(q)
    elif fn == "ceil":
        k = math.ceil(q)
    elif fn == "round":
        k = math.floor(abs(q) + Fraction(1, 2))
        k = -k if q < 0 else k
    else:                                             # rint: ties to even
        k = round(q)
    v = math.copysign(float(k), x)
    return v, v, 0.0


def evaluate1(fn, fmt_name, x, y=None):
    """Correctly rounded fn(x) (or fn(x, y)) in format ``fmt_name``.

    Binary functions take their arguments in C order: pow(x, y),
    atan2(x=y_c, y=x_c) -- i.e. evaluate1("atan2", f, a, b) is atan2(a, b) --
    fmod(x, y) and remainder(x, y).  Arguments are Python floats holding
    values of that format (binary64 for 'f64', binary32 values for 'f32', and
    so on).  Returns (rn, hi, lo): the
    rounded result and a binary64 pair approximating the exact value (equal to
    (rn, 0) when the result is exact or special)."""
    fmt = FORMATS[fmt_name]
    prec0 = fmt.p + 40
    if fn in EXACT_UNARY:
        return _exact_unary(fn, x, fmt, prec0)
    if fn in UNARY:
        sp = _special_unary(fn, x)
        if sp is not None:
            return sp, sp, 0.0
        if fn == "exp2" and _is_int(x):
            k = int(max(-5000.0, min(5000.0, x)))
            v = rn_dyadic(1, k, fmt)
            return v, v, 0.0
        if fn == "log2":
            m, e = _dyadic(x)
            if m == 1:
                v = rn_dyadic(e, 0, fmt, zero_sign=1)
                return v, v, 0.0
        if fn == "atan" and math.isinf(x):
            v = math.copysign(_round_const("pi/2", fmt), x)
            return v, v, 0.0
        if fn == "acos" and x == -1.0:
            v = _round_const("pi", fmt)
            return v, v, 0.0
        if fn == "log10":
            m, e = _dyadic(x)
            if e > 0 and m == 5 ** e:                 # x = 10^e
                v = rn_dyadic(e, 0, fmt)
                return v, v, 0.0
        if fn == "exp10" and _is_int(x) and x > 0:
            return _exact_result(10 ** int(min(x, 400.0)), 0, fmt)
        if fn == "erf" and abs(x) > 27.0:
            # 1 - erf|x| < 2^-1050: the result is +-1 in every format, and
            # so is the exact value to far below any ulp
            v = math.copysign(1.0, x)
            return v, v, 0.0
        if fn == "erfc" and abs(x) > 28.0:
            # erfc x < 2^-1135 (x > 28) or 2 - that: +0 or 2 in every format
            v = 0.0 if x > 0 else 2.0
            return v, v, 0.0
        if fn == "cbrt":
            ex = _cbrt_exact(x)
            if ex is not None:
                return _exact_result(ex[0] if x > 0 else -ex[0], ex[1], fmt)
        if fn == "tgamma":
            if x > 200.0:                             # Gamma(200) > 2^1240: +inf
                return INF, INF, 0.0
            if x == math.floor(x):                    # Gamma(n) = (n - 1)!
                return _exact_result(math.factorial(int(x) - 1), 0, fmt)
            if x < -200.0:
                # |Gamma(x)| < 2^-1190 here: a zero with the sign of sin(pi x)
                v = 0.0 if math.floor(x) % 2 == 0 else -0.0
                return v, v, 0.0
        return _ziv(_BALLS[fn], (x,), fmt, prec0)
    if fn == "atan2":
        sp = _special_atan2(x, y, fmt)       # atan2(x, y) in C order
        if sp is not None:
            return sp, sp, 0.0
        return _ziv(_ball_atan2, (x, y), fmt, prec0)
    if fn == "pow":
        sp = _special_pow(x, y)
        if sp is not None:
            return sp, sp, 0.0
        neg = x < 0 and _is_odd_int(y)
        ex = _pow_exact(x, y)
        if ex is not None:
            m, e = ex
            return _exact_result(-m if neg else m, e, fmt, zero_sign=-1 if neg else 1)
        v, hi, lo = _ziv(_ball_pow, (x, y), fmt, prec0)
        if neg:
            return -v, -hi, -lo
        return v, hi, lo
    if fn == "hypot":
        sp = _special_hypot(x, y)
        if sp is not None:
            return sp, sp, 0.0
        if x == 0.0 and y == 0.0:
            return 0.0, 0.0, 0.0
        S, e = _sum_squares(x, y)
        r = math.isqrt(S)
        if r * r == S:                                # also |x| when y = 0
            return _exact_result(r, e // 2, fmt)
        return _ziv(_ball_hypot, (x, y), fmt, prec0)
    if fn == "fdim":
        if math.isnan(x) or math.isnan(y):
            return NAN, NAN, 0.0
        if not x > y:
            return 0.0, 0.0, 0.0
        if math.isinf(x) or math.isinf(y):            # x = +inf or y = -inf
            return INF, INF, 0.0
        (nx, dx), (ny, dy) = x.as_integer_ratio(), y.as_integer_ratio()
        d = max(dx, dy)                               # powers of two
        num = nx * (d // dx) - ny * (d // dy)
        v = rn_dyadic(num, -(d.bit_length() - 1), fmt)
        return v, v, 0.0
    if fn == "copysign":
        v = math.copysign(x, y)
        return v, v, 0.0
    if fn == "nextafter":
        if math.isnan(x) or math.isnan(y):
            return NAN, NAN, 0.0
        if fmt_name == "f64":
            v = math.nextafter(x, y)
        elif fmt_name == "f32":
            import numpy as np
            v = float(np.nextafter(np.float32(x), np.float32(y)))
        else:
            raise ValueError("nextafter: binary64 and binary32 only")
        return v, v, 0.0
    if fn in ("fmax", "fmin"):
        if math.isnan(x):
            return y, y, 0.0
        if math.isnan(y):
            return x, x, 0.0
        # order: -0 before +0; otherwise the numeric order
        kx = (x, math.copysign(1.0, x))
        ky = (y, math.copysign(1.0, y))
        v = (x if kx >= ky else y) if fn == "fmax" else (x if kx <= ky else y)
        return v, v, 0.0
    if fn in ("fmod", "remainder"):
        sp = _special_fmod(x, y)
        if sp is not None:
            return sp, sp, 0.0
        r, e = _fmod_exact(x, y, fn == "remainder")
        if r == 0:
            v = math.copysign(0.0, x)
        else:
            v = rn_dyadic(r if x > 0 else -r, e, fmt)
        return v, v, 0.0
    raise ValueError("unknown function %r" % fn)
