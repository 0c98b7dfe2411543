"""Pins of the oracle's gamma function and its logarithm (oracle/gamma.py)
against what mathematics fixes, independently of its Stirling-series path:

* Gamma(n) = (n - 1)! for positive integers, through the ball path (not the
  exact shortcut);
* the recurrence Gamma(x + 1) = x Gamma(x), the reflection formula
  Gamma(x) Gamma(1 - x) = pi / sin(pi x) on (0, 1) (both sides through the
  positive-argument path) and Legendre's duplication formula
  Gamma(x) Gamma(x + 1/2) = 2^(1 - 2x) sqrt(pi) Gamma(2x), as ball identities;
* exact points and the C99 Annex F special values;
* mpmath (high precision, tests only) and the host C library's lgamma/tgamma
  (within its few ulps) on random arguments of both signs.
"""
import math
import random

import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import ball as B
from oracle.consts import pi
from oracle.elementary import log_ball, log_of_ball, sin_cos_ball
from oracle.gamma import lgamma_ball, tgamma_ball, bernoulli_even
from fractions import Fraction


def _contains_zero(b):
    return abs(b.m) <= b.r


def test_bernoulli_numbers():
    b = bernoulli_even(6)
    assert b == [Fraction(1, 6), Fraction(-1, 30), Fraction(1, 42), Fraction(-1, 30),
                 Fraction(5, 66), Fraction(-691, 2730)]


@pytest.mark.parametrize("n", list(range(1, 41)) + [100, 170])
def test_gamma_of_integers_through_the_ball_path(n):
    g = tgamma_ball(float(n), 120)
    f = math.factorial(n - 1)
    lo, hi, e = g.lo_hi()
    # the exact factorial lies inside the ball
    assert Fraction(lo) * Fraction(2) ** e <= f <= Fraction(hi) * Fraction(2) ** e


def _ball_check(expr):
    assert _contains_zero(expr), expr


def test_recurrence_reflection_duplication():
    rng = random.Random(7)
    P = 160
    for _ in range(60):
        x = rng.uniform(0.01, 60.0)
        if x == math.floor(x):
            continue
        # Gamma(x + 1) = x Gamma(x)
        m, e = Fraction(x).numerator, -(Fraction(x).denominator.bit_length() - 1)
        exact1 = Fraction(x + 1.0) == Fraction(x) + 1
        lhs = B.sub(lgamma_ball(x + 1.0, P), lgamma_ball(x, P), P) if exact1 else None
        if lhs is not None:
            _ball_check(B.sub(lhs, log_ball(m, e, P), P))
        # duplication: lG(x) + lG(x + 1/2) = (1 - 2x) ln 2 + ln(pi)/2 + lG(2x)
        if Fraction(x + 0.5) == Fraction(x) + Fraction(1, 2):
            l = B.add(lgamma_ball(x, P), lgamma_ball(x + 0.5, P), P)
            ln2 = log_ball(2, 0, P)
            r = B.add(B.mul(B.sub(B.exact(1), B.from_float(2 * x), P), ln2, P),
                      B.scale2(log_of_ball(pi(P), P), -1), P)
            r = B.add(r, lgamma_ball(2 * x, P), P)
            _ball_check(B.sub(l, r, P))
    for _ in range(40):
        x = rng.uniform(0.001, 0.999)
        if Fraction(1.0 - x) != 1 - Fraction(x):
            continue
        # reflection on (0, 1): lG(x) + lG(1 - x) = ln pi - ln sin(pi x)
        l = B.add(lgamma_ball(x, P), lgamma_ball(1.0 - x, P), P)
        s, _ = sin_cos_ball(B.mul(pi(P + 8), B.from_float(x if x <= 0.5 else 1.0 - x), P), P)
        r = B.sub(log_of_ball(pi(P), P), log_of_ball(s, P), P)
        _ball_check(B.sub(l, r, P))


def test_exact_points_and_annex_f():
    ev = lambda fn, xs: oracle.evaluate(fn, "f64", np.array(xs, dtype=np.float64))[0]
    v = ev("lgamma", [1.0, 2.0, 3.0, 0.0, -0.0, -1.0, -7.0, np.inf, -np.inf, np.nan])
    assert v[0] == 0.0 and v[1] == 0.0 and not math.copysign(1, v[0]) < 0
    assert v[2] == math.log(2.0)
    assert np.all(np.isinf(v[3:9]) & (v[3:9] > 0)) and np.isnan(v[9])
    v = ev("tgamma", [1.0, 5.0, 171.0, 172.0, 0.0, -0.0, -1.0, -1e300, np.inf, -np.inf, np.nan])
    assert v[0] == 1.0 and v[1] == 24.0 and v[2] == float(math.factorial(170))
    assert v[3] == np.inf and v[4] == np.inf and v[5] == -np.inf
    assert np.isnan(v[6]) and np.isnan(v[7]) and v[8] == np.inf and np.isnan(v[9])
    assert np.isnan(v[10])


def _mp_round(v, fmt):
    if fmt == "f64":
        return float(v)
    # binary32: round the high-precision value once (overflow: at or beyond
    # the midpoint between the largest float and 2^128)
    if abs(v) >= mp.mpf(2) ** 128 * (1 - mp.mpf(2) ** -25):
        return math.copysign(math.inf, float(v))
    with mp.workprec(24):
        return float(+v) if abs(v) >= mp.mpf(2) ** -126 else float(mp.nint(v * 2 ** 149) / 2 ** 149)


@pytest.mark.parametrize("fmt", ["f64", "f32"])
@pytest.mark.parametrize("fn", ["lgamma", "tgamma"])
def test_against_mpmath(fn, fmt):
    rng = np.random.default_rng(91 + len(fn) + len(fmt))
    xs = np.concatenate([rng.uniform(-30, 30, 150), np.exp(rng.uniform(-40, 5, 50)),
                         -np.exp(rng.uniform(-40, 3, 50)), rng.uniform(0.5, 2.5, 50)])
    if fmt == "f32":
        xs = xs.astype(np.float32).astype(np.float64)
    xs = xs[xs != np.floor(xs)]
    rn, hi, lo = oracle.evaluate(fn, fmt, xs)
    mp.mp.prec = 400
    for x, r, h, l in zip(xs, rn, hi, lo):
        g = mp.gamma(mp.mpf(float(x)))
        want = mp.log(abs(g)) if fn == "lgamma" else g
        assert r == _mp_round(want, fmt), (fn, fmt, x, r, want)
        if want != 0:
            tol = mp.mpf(2) ** (-90 if fmt == "f64" else -60)    # the oracle's p + 40 bits
            assert abs((mp.mpf(h) + mp.mpf(l)) - want) <= abs(want) * tol, x


def test_against_the_host_c_library():
    """Python's math.lgamma / math.gamma: an independent implementation,
    within a few binary64 ulps away from the lgamma zeros."""
    rng = np.random.default_rng(5)
    xs = np.concatenate([rng.uniform(0.01, 150, 300), -rng.uniform(0.01, 150, 300)])
    xs = xs[xs != np.floor(xs)]
    rl = oracle.evaluate("lgamma", "f64", xs)[0]
    rt = oracle.evaluate("tgamma", "f64", xs)[0]
    for x, a, b in zip(xs, rl, rt):
        la = math.lgamma(x)
        if abs(la) > 1.0:
            assert abs(a - la) <= 16 * math.ulp(la), (x, a, la)
        if abs(x) < 170:
            ga = math.gamma(x)
            assert abs(b - ga) <= 32 * math.ulp(ga), (x, b, ga)
