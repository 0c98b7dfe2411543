"""Correctly rounded products g * f'(x) for the backward kernels.

Test infrastructure only.  The derivatives are the textbook ones:

    sin' = cos, cos' = -sin, tan' = 1 / cos^2, exp' = exp, log' = 1 / x,
    tanh' = 1 / cosh^2,
    d/dx x^y = y x^(y-1),  d/dy x^y = x^y log x   (x > 0),
    d/dy atan2(y, x) = x / (x^2 + y^2),  d/dx atan2(y, x) = -y / (x^2 + y^2).

Each is evaluated as a ball times the exact upstream gradient g and rounded
once (Ziv), like the forward functions.  Arguments must be finite with a
finite, nonzero derivative; callers filter the rest.
"""
import math

from . import ball as B
from .ball import exact, from_float, mul, div, add, sub
from .elementary import sincos_reduced, sin_cos_ball, exp_ball, log_ball, sinh_cosh_small
from .functions import _ziv, _dyadic, _clamp_exp_arg
from .rounding import FORMATS

__all__ = ["grad1", "grad_pow", "grad_atan2"]


def _cos_sin(x, prec):
    m, e = _dyadic(x)
    k, r = sincos_reduced(m, e, prec)
    s, c = sin_cos_ball(r, prec + 8)
    sin_b = (s, c, B.neg(s), B.neg(c))[k]
    cos_b = (c, B.neg(s), B.neg(c), s)[k]
    return sin_b, cos_b


def _cosh_ball(x, prec):
    ax = abs(x)
    if ax < 1.0:
        return sinh_cosh_small(from_float(ax), prec)[1]
    E = exp_ball(_clamp_exp_arg(from_float(ax)), prec + 8)
    return B.scale2(add(E, div(exact(1), E, prec + 8), prec + 8), -1)


def _g_sin(x, g, prec):
    return mul(_cos_sin(x, prec)[1], from_float(g), prec)


def _g_cos(x, g, prec):
    return B.neg(mul(_cos_sin(x, prec)[0], from_float(g), prec))


def _g_tan(x, g, prec):
    c = _cos_sin(x, prec + 8)[1]
    return div(from_float(g), mul(c, c, prec + 8), prec)


def _g_exp(x, g, prec):
    return mul(exp_ball(_clamp_exp_arg(from_float(x)), prec + 8), from_float(g), prec)


def _g_log(x, g, prec):
    return div(from_float(g), from_float(x), prec)


def _g_tanh(x, g, prec):
    c = _cosh_ball(x, prec + 8)
    return div(from_float(g), mul(c, c, prec + 8), prec)


_G = {"sin": _g_sin, "cos": _g_cos, "tan": _g_tan, "exp": _g_exp, "log": _g_log,
      "tanh": _g_tanh}


def grad1(fn, fmt_name, x, g):
    """RN(g * fn'(x)) and the (hi, lo) pair, for finite x and g."""
    fmt = FORMATS[fmt_name]
    if g == 0.0:
        return 0.0, 0.0, 0.0
    return _ziv(_G[fn], (x, g), fmt, fmt.p + 40)


def _pow_ball(x, yb, prec):
    """x^Y for x > 0 and an exact ball exponent Y; also returns log x."""
    m, e = _dyadic(x)
    L = log_ball(m, e, prec + 40)
    return exp_ball(_clamp_exp_arg(mul(L, yb, prec + 40)), prec + 8), L


def _g_pow_x(x, y, g, prec):
    ym1 = B.sub(from_float(y), exact(1), 4 * prec)          # y - 1, exact
    p, _ = _pow_ball(x, ym1, prec)
    return mul(mul(p, from_float(y), prec + 8), from_float(g), prec)


def _g_pow_y(x, y, g, prec):
    p, L = _pow_ball(x, from_float(y), prec)
    return mul(mul(p, L, prec + 8), from_float(g), prec)


def grad_pow(fmt_name, x, y, g):
    """(RN(g y x^(y-1)), RN(g x^y log x)) for finite x > 0, finite y, g."""
    fmt = FORMATS[fmt_name]
    if g == 0.0:
        z = (0.0, 0.0, 0.0)
        return z, z
    gx = _ziv(_g_pow_x, (x, y, g), fmt, fmt.p + 40)
    gy = (0.0, 0.0, 0.0) if x == 1.0 else _ziv(_g_pow_y, (x, y, g), fmt, fmt.p + 40)
    return gx, gy


def _g_atan2_y(y, x, g, prec):
    d = add(mul(from_float(x), from_float(x), prec + 8),
            mul(from_float(y), from_float(y), prec + 8), prec + 8)
    return div(mul(from_float(x), from_float(g), prec + 8), d, prec)


def _g_atan2_x(y, x, g, prec):
    d = add(mul(from_float(x), from_float(x), prec + 8),
            mul(from_float(y), from_float(y), prec + 8), prec + 8)
    return B.neg(div(mul(from_float(y), from_float(g), prec + 8), d, prec))


def grad_atan2(fmt_name, y, x, g):
    """(d/dy, d/dx) of atan2(y, x) times g, correctly rounded; (y, x) != 0."""
    fmt = FORMATS[fmt_name]
    z = (0.0, 0.0, 0.0)
    if g == 0.0:
        return z, z
    gy = z if x == 0.0 else _ziv(_g_atan2_y, (y, x, g), fmt, fmt.p + 40)
    gx = z if y == 0.0 else _ziv(_g_atan2_x, (y, x, g), fmt, fmt.p + 40)
    return gy, gx
