"""The array IEEE remainder of tests/exact_ref.py against the C library's
remainder (Python's math.remainder), element by element."""
import math

import numpy as np

from tests.exact_ref import ieee_remainder


def _same(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return (a == b) & (np.signbit(a) == np.signbit(b)) | (np.isnan(a) & np.isnan(b))


def _host(x, y):
    return np.array([math.remainder(a, b) if not (math.isnan(a) or math.isnan(b) or math.isinf(a)
                                                 or b == 0.0) else math.nan
                     for a, b in zip(x.tolist(), y.tolist())])


def test_random_magnitudes():
    rng = np.random.default_rng(5)
    n = 200000
    x = np.sign(rng.standard_normal(n)) * 10.0 ** rng.uniform(-300, 300, n)
    y = np.sign(rng.standard_normal(n)) * 10.0 ** rng.uniform(-300, 300, n)
    assert _same(ieee_remainder(x, y), _host(x, y)).all()


def test_ties_extremes_and_specials():
    big = np.finfo(np.float64).max
    tiny = 5e-324
    vals = [0.0, -0.0, tiny, -tiny, 1.0, -1.0, 0.5, 1.5, 2.5, -2.5, 3.0, 4.5, 1e308, -1e308, big,
            -big, 2.0 ** -1022, 3 * tiny, math.inf, -math.inf, math.nan]
    x = np.array([a for a in vals for _ in vals])
    y = np.array([b for _ in vals for b in vals])
    # exact ties: x = (k + 1/2) y
    k = np.arange(-40, 41, dtype=np.float64)
    x = np.concatenate([x, (k + 0.5) * 0.75, (k + 0.5) * 3.0 * tiny, (k + 0.5) * 2.0 ** 1000])
    y = np.concatenate([y, np.full(k.size, 0.75), np.full(k.size, 3.0 * tiny),
                        np.full(k.size, 2.0 ** 1000)])
    got = ieee_remainder(x, y)
    want = _host(x, y)
    bad = ~_same(got, want)
    assert not bad.any(), (x[bad][:4], y[bad][:4], got[bad][:4], want[bad][:4])


def test_binary32_operands():
    rng = np.random.default_rng(6)
    n = 100000
    x = (np.sign(rng.standard_normal(n)) * 10.0 ** rng.uniform(-38, 38, n)).astype(np.float32)
    y = (np.sign(rng.standard_normal(n)) * 10.0 ** rng.uniform(-38, 38, n)).astype(np.float32)
    got = ieee_remainder(x, y).astype(np.float32)
    want = _host(x.astype(np.float64), y.astype(np.float64)).astype(np.float32)
    assert _same(got, want).all()
