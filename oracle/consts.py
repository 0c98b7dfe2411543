"""Mathematical constants as rigorous balls, computed from series.

Test infrastructure only: nothing in the library path may import this module.

* pi by Machin's formula, pi = 16 atan(1/5) - 4 atan(1/239), in fixed point.
* ln 2 by 2 atanh(1/3) = 2 * sum 1 / ((2k+1) 3^(2k+1)).

The paper's Payne-Hanek table needs 2/pi to about 1280 bits (Appendix A,
table generator); the oracle's reduction asks for as many bits as the
argument's exponent requires and recomputes at a higher precision on demand.
Both constants are pinned in the tests against an independent algorithm
(Gauss-Legendre AGM for pi, a different series for ln 2) and the paper's
printed double-double constants for pi/2 and 2 pi.
"""
from .ball import Ball, div, exact

__all__ = ["pi", "ln2", "two_over_pi", "half_pi"]

_GUARD = 40


def _atan_inv_fixed(n, bits):
    """floor-ish of atan(1/n) * 2**bits with a bound on the error in units.

    Every summand is truncated at most twice (the power and the division by
    2k+1); each truncation error is < 1 unit and the truncated power carries
    at most 2 units of error from the previous ones, so a summand is off by
    < 3 units.  The alternating tail after the last summand is smaller than
    the first omitted one, which is < 1 unit when the loop stops."""
    one = 1 << bits
    n2 = n * n
    power = one // n
    total = power
    k = 1
    sign = -1
    terms = 1
    while power:
        power //= n2
        t = power // (2 * k + 1)
        total += sign * t
        sign = -sign
        k += 1
        terms += 1
    return total, 3 * terms + 1


_cache = {}


def pi(prec):
    """Ball containing pi, with at least ``prec`` correct bits."""
    key = ("pi", prec)
    if key not in _cache:
        bits = prec + _GUARD
        a, ea = _atan_inv_fixed(5, bits)
        b, eb = _atan_inv_fixed(239, bits)
        _cache[key] = Ball(16 * a - 4 * b, 16 * ea + 4 * eb, -bits)
    return _cache[key]


def ln2(prec):
    """Ball containing ln 2 = 2 atanh(1/3)."""
    key = ("ln2", prec)
    if key not in _cache:
        bits = prec + _GUARD
        one = 1 << bits
        power = one // 3          # 3^-(2k+1) in fixed point
        total = power
        k = 1
        terms = 1
        while power:
            power //= 9
            total += power // (2 * k + 1)
            k += 1
            terms += 1
        _cache[key] = Ball(2 * total, 2 * (3 * terms + 1), -bits)
    return _cache[key]


def two_over_pi(prec):
    key = ("2/pi", prec)
    if key not in _cache:
        _cache[key] = div(exact(2), pi(prec + 8), prec + 4)
    return _cache[key]


def half_pi(prec):
    p = pi(prec)
    return Ball(p.m, p.r, p.e - 1)
