"""The gamma function and its logarithm, as rigorous balls.

Test infrastructure only: nothing in the library path may import this module.

C99's tgamma and lgamma belong to the real function set the paper's library
provides (Section 1); the paper does not describe them.  These are textbook
definitions, chosen to be checked by eye:

* log Gamma(z) for z > 0: shift up, z + N = w with w at least W (the
  recurrence Gamma(z + 1) = z Gamma(z) gives
  log Gamma(z) = log Gamma(w) - log(z (z + 1) ... (z + N - 1)), the product
  an exact dyadic), then Stirling's series
  log Gamma(w) = (w - 1/2) log w - w + log(2 pi)/2
                 + sum_{k=1..K} B_2k / (2k (2k - 1) w^(2k - 1)) + R_K,
  |R_K| <= |B_(2K+2)| / ((2K + 2)(2K + 1) w^(2K + 1))  (w > 0 real),
  with B_2k the Bernoulli numbers (exact rationals).  The truncation bound is
  added to the ball.
* z < 0, not an integer: the reflection formula
  Gamma(z) Gamma(1 - z) = pi / sin(pi z), so
  log|Gamma(z)| = log pi - log|sin(pi z)| - log Gamma(1 - z), sin(pi z) from
  the exact fraction f = z - round(z) (|f| <= 1/2): sin(pi z) = (-1)^round(z)
  sin(pi f).
* Gamma(z) = sign * exp(log|Gamma(z)|), the sign that of sin(pi z) for z < 0.

Exact cases (where Ziv's loop would not end): Gamma(n) = (n - 1)! for
positive integers n, log Gamma(1) = log Gamma(2) = 0.  Every other finite
result is irrational (for dyadic z not an integer, Gamma(z) is not a dyadic
rational... the loop just needs it not to be exactly representable or a
midpoint, which the tests confirm on their sample by termination).
"""
import math
from fractions import Fraction

from . import ball as B
from .ball import exact, add, sub, mul, div, mag_log2
from .consts import pi
from .elementary import exp_ball, log_ball, log_of_ball, sin_cos_ball, tail_ball

__all__ = ["lgamma_ball", "tgamma_ball", "bernoulli_even"]

_BERN = [Fraction(1)]          # B_0, B_1, B_2, ... (B_1 = -1/2)


def _bernoulli(n):
    """B_0 .. B_n by the recurrence sum_{j=0}^{m} C(m+1, j) B_j = 0."""
    while len(_BERN) <= n:
        m = len(_BERN)
        s = Fraction(0)
        c = 1                                   # C(m+1, j), j = 0
        for j in range(m):
            s += c * _BERN[j]
            c = c * (m + 1 - j) // (j + 1)
        _BERN.append(-s / (m + 1))
    return _BERN


def bernoulli_even(k):
    """B_2, B_4, ..., B_2k as exact fractions."""
    b = _bernoulli(2 * k + 2)
    return [b[2 * i] for i in range(1, k + 1)]


def _frac_ball(q, prec):
    return div(exact(q.numerator), exact(q.denominator), prec)


def _log_gamma_shifted(w, wp):
    """Stirling's series for a ball w >= 8 (dyadic, exact), as a ball."""
    lw = log_of_ball(w, wp)
    s = sub(mul(sub(w, exact(1, -1), wp), lw, wp), w, wp)
    l2pi = log_of_ball(B.scale2(pi(wp + 8), 1), wp)
    s = add(s, B.scale2(l2pi, -1), wp)
    inv = div(exact(1), w, wp)
    inv2 = mul(inv, inv, wp)
    p = inv                                            # 1 / w^(2k-1)
    k = 1
    while True:
        b = _bernoulli(2 * k + 2)
        t = mul(_frac_ball(b[2 * k] / (2 * k * (2 * k - 1)), wp), p, wp)
        s = add(s, t, wp)
        p = mul(p, inv2, wp)
        # bound of the remainder after term k: |B_(2k+2)| / ((2k+2)(2k+1) w^(2k+1))
        nxt = abs(b[2 * k + 2]) / ((2 * k + 2) * (2 * k + 1))
        bound = mag_log2(_frac_ball(nxt, 64)) + mag_log2(p)
        if bound < -wp - 8 or k > 400:
            return tail_ball(s, bound)
        k += 1


def _lgamma_positive(z, prec):
    """log Gamma(z) for an exact positive z (a Fraction with power-of-two
    denominator)."""
    wp = prec + 24
    W = max(12, wp // 4)
    N = 0 if z >= W else int(math.ceil(W - z))
    w = z + N
    wb = div(exact(w.numerator), exact(w.denominator), wp)
    s = _log_gamma_shifted(wb, wp)
    if N:
        prod = Fraction(1)
        for i in range(N):
            prod *= z + i
        den = prod.denominator
        e = -(den.bit_length() - 1)
        assert den == 1 << -e
        s = sub(s, log_ball(prod.numerator, e, wp), wp)
    return s


def _sin_pi(z, prec):
    """sin(pi z) for an exact z that is not an integer, as a ball."""
    n = math.floor(z + Fraction(1, 2))
    f = z - n                                          # |f| <= 1/2, exact
    wp = prec + 16
    r = mul(pi(wp), _frac_ball(f, wp + 8), wp)         # |r| <= pi/2
    s, _ = sin_cos_ball(r, wp)
    return B.neg(s) if n % 2 else s


def lgamma_ball(x, prec):
    """log|Gamma(x)| for a finite binary float x that is not zero or a
    negative integer."""
    z = Fraction(x)
    if z > 0:
        return _lgamma_positive(z, prec)
    wp = prec + 24
    sp = _sin_pi(z, wp)
    lsin = log_of_ball(B.Ball(abs(sp.m), sp.r, sp.e), wp)
    lpi = log_of_ball(pi(wp), wp)
    return sub(sub(lpi, lsin, wp), _lgamma_positive(1 - z, wp), wp)


def tgamma_ball(x, prec):
    """Gamma(x) for a finite binary float x that is not zero or a negative
    integer, with |log|Gamma(x)|| < 2100 (callers treat the rest)."""
    wp = prec + 16
    lg = lgamma_ball(x, wp + 16)
    g = exp_ball(lg, wp)
    if x < 0:
        sp = _sin_pi(Fraction(x), 64)
        if B.contains_zero(sp):
            raise B.PrecisionError("sign of sin(pi x) undecided")
        if B.is_negative(sp):
            g = B.neg(g)
    return g
