"""IEEE remainder over whole arrays, exact, for the full-size checks.

remainder(x, y) = x - n y with n the integer nearest x / y, ties to even
(C99 7.12.10.2; the paper's "FP Remainder", Section 5).  With d = |y| and
r = fmod(x, 2d) (exact, the sign of x, |r| < 2d, and x = 2 q d + r for an
integer q), the nearest integer to x / d is 2q + m with m in {0, 1, 2}
chosen from |r| against d/2 and 3d/2; ties pick the even total, that is
m = 0 at |r| = d/2 and m = 2 at |r| = 3d/2.  The comparisons and r - m d run
in the host's 80-bit extended format, where 2|r|, 3d and r - m d are exact
(64-bit significands, a wider exponent range); the result is a binary64
value, so the final conversion is exact too.  A zero result takes the sign
of x.  Checked against the C library's remainder in
tests/test_exact_ref.py.
"""
import concurrent.futures as cf

import numpy as np


def _chunked(f, x, y, threads=16, chunk=1 << 20):
    """f over [x, y] in chunks on a thread pool (numpy's ufuncs release the
    interpreter lock; the host fmod takes time linear in the exponent gap)."""
    x = np.asarray(x)
    y = np.asarray(y)
    if x.size <= chunk:
        return f(x, y)
    out = [None] * ((x.size + chunk - 1) // chunk)
    with cf.ThreadPoolExecutor(threads) as ex:
        futs = {ex.submit(f, x[s:s + chunk], y[s:s + chunk]): i
                for i, s in enumerate(range(0, x.size, chunk))}
        for fu, i in futs.items():
            out[i] = fu.result()
    return np.concatenate(out)


def fmod(x, y):
    """The host C library's fmod (exact) over whole arrays, in parallel."""
    return _chunked(np.fmod, x, y)


def ieee_remainder(x, y):
    """IEEE remainder of whole arrays (binary64 result), in parallel."""
    return _chunked(_remainder, x, y)


def _remainder(x, y):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = np.abs(y)
    with np.errstate(all="ignore"):
        r = np.fmod(x, 2.0 * d)                     # 2d = inf: fmod gives x, |x| < 2d
        R = np.abs(r).astype(np.longdouble) * 2
        D = d.astype(np.longdouble)
        m = np.where(R <= D, 0, np.where(R < 3 * D, 1, 2)).astype(np.longdouble)
        adj = r.astype(np.longdouble) - np.sign(r).astype(np.longdouble) * m * D
        res = np.where(m == 0, r, adj.astype(np.float64))
    res = np.where(res == 0.0, np.copysign(0.0, x), res)
    return res
