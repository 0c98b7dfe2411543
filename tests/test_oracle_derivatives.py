"""Pins for the oracle's derivative products g * f'(x): against mpmath's
numerical differentiation (mp.diff, which knows no derivative formula) at 300
bits, rounded to the output format."""
import random

import mpmath
import pytest

from oracle.derivatives import grad1, grad_pow, grad_atan2

F = {"sin": mpmath.sin, "cos": mpmath.cos, "tan": mpmath.tan, "exp": mpmath.exp,
     "log": mpmath.log, "tanh": mpmath.tanh}


@pytest.mark.parametrize("fn", sorted(F))
def test_unary_derivatives_vs_numerical_differentiation(fn):
    rng = random.Random(len(fn))
    for _ in range(60):
        x = rng.uniform(0.1, 10.0)
        g = rng.uniform(-3, 3)
        got = grad1(fn, "f64", x, g)[0]
        with mpmath.workprec(300):
            d = mpmath.diff(F[fn], mpmath.mpf(x))
            want = float(d * mpmath.mpf(g))
        assert got == want, (fn, x, g, got, want)


def test_pow_and_atan2_partials_vs_numerical_differentiation():
    rng = random.Random(3)
    for _ in range(60):
        x = rng.uniform(0.1, 10.0)
        y = rng.uniform(0.1, 10.0)
        g = rng.uniform(-3, 3)
        (gx, _, _), (gy, _, _) = grad_pow("f64", x, y, g)
        with mpmath.workprec(300):
            X, Y, G = mpmath.mpf(x), mpmath.mpf(y), mpmath.mpf(g)
            wx = float(G * mpmath.diff(lambda t: mpmath.power(t, Y), X))
            wy = float(G * mpmath.diff(lambda t: mpmath.power(X, t), Y))
        assert gx == wx and gy == wy, (x, y, g)
        (ay, _, _), (ax, _, _) = grad_atan2("f64", y, x, g)
        with mpmath.workprec(300):
            wy = float(G * mpmath.diff(lambda t: mpmath.atan2(t, X), Y))
            wx = float(G * mpmath.diff(lambda t: mpmath.atan2(Y, t), X))
        assert ay == wy and ax == wx, (y, x, g)
