"""Minimax polynomial coefficients by the Remez exchange algorithm.

The paper generates its polynomial coefficients with its own tool that
minimises the maximum relative error, with the lowest-order terms kept in
higher precision (Section 5, "Overview of Library Implementation").  This is
that tool for this library, written from the textbook algorithm:

    minimise  max_{z in [a, b]} | w(z) * (f(z) - sum_i c_i z^i) |

1. start from the Chebyshev extrema of [a, b] as the reference set;
2. solve the linear system that makes the weighted error equioscillate with
   level E on the reference;
3. locate the extrema of the error function (dense Chebyshev grid, then a
   golden-section refinement) and exchange the reference;
4. stop when the largest error equals |E| to a relative 1e-6.

Rounding the coefficients to the target format is done greedily: the lowest
free coefficient is rounded (to a double, a float, or kept as a hi+lo pair),
then the remaining ones are re-optimised with it fixed, and so on upwards.
The reported error is that of the rounded polynomial, evaluated exactly.

All arithmetic is mpmath at 320 bits; this module is a build step only.
"""
import mpmath as mp

__all__ = ["remez", "remez_rounded", "max_error", "round_to"]

mp.mp.prec = 320


def _cheb_points(a, b, n):
    return [(a + b) / 2 - (b - a) / 2 * mp.cos(mp.pi * j / (n - 1)) for j in range(n)]


def _poly(c, z):
    s = mp.mpf(0)
    for ci in reversed(c):
        s = s * z + ci
    return s


def _solve(f, w, ref, n, fixed):
    """Coefficients c_k for k not in fixed, plus the level E."""
    free = [k for k in range(n) if k not in fixed]
    m = len(free)
    A = mp.matrix(m + 1, m + 1)
    rhs = mp.matrix(m + 1, 1)
    for j, z in enumerate(ref):
        for col, k in enumerate(free):
            A[j, col] = z ** k
        A[j, m] = (-1) ** j / w(z)
        rhs[j] = f(z) - sum(fixed[k] * z ** k for k in fixed)
    sol = mp.lu_solve(A, rhs)
    c = [None] * n
    for k in fixed:
        c[k] = fixed[k]
    for col, k in enumerate(free):
        c[k] = sol[col]
    return c, sol[m]


def _golden_max(g, lo, hi, iters=60):
    """Maximise |g| on [lo, hi] (unimodal near an extremum)."""
    gr = (mp.sqrt(5) - 1) / 2
    a, b = lo, hi
    c = b - gr * (b - a)
    d = a + gr * (b - a)
    fc, fd = abs(g(c)), abs(g(d))
    for _ in range(iters):
        if fc > fd:
            b, d, fd = d, c, fc
            c = b - gr * (b - a)
            fc = abs(g(c))
        else:
            a, c, fc = c, d, fd
            d = a + gr * (b - a)
            fd = abs(g(d))
    z = (a + b) / 2
    return z, g(z)


def _extrema(err, a, b, m, grid):
    zs = _cheb_points(a, b, grid)
    es = [err(z) for z in zs]
    # runs of constant sign; the extremum of each run
    runs = []
    start = 0
    for i in range(1, len(zs) + 1):
        if i == len(zs) or mp.sign(es[i]) != mp.sign(es[start]):
            seg = range(start, i)
            k = max(seg, key=lambda t: abs(es[t]))
            runs.append(k)
            start = i
    pts = []
    for k in runs:
        lo = zs[max(k - 1, 0)]
        hi = zs[min(k + 1, len(zs) - 1)]
        if k == 0 or k == len(zs) - 1:
            pts.append((zs[k], es[k]))
        else:
            pts.append(_golden_max(err, lo, hi))
    # keep m points with alternating signs and the largest magnitudes
    while len(pts) > m:
        # drop the smaller end, or merge the weakest interior pair
        if abs(pts[0][1]) < abs(pts[-1][1]):
            pts.pop(0)
        else:
            pts.pop()
    return pts


def _away_from_weight_zeros(ref, w, a, b):
    """A reference point where the weight (nearly) vanishes carries no
    information -- the weighted error is zero there -- and makes the system
    singular: nudge such points aside."""
    ws = [abs(w(z)) for z in ref]
    top = max(ws)
    out = []
    for z, wz in zip(ref, ws):
        if wz < top * mp.mpf("1e-12"):
            z = z + (b - a) * mp.mpf("1e-3") if z + (b - a) * mp.mpf("1e-3") <= b \
                else z - (b - a) * mp.mpf("1e-3")
        out.append(z)
    return out


def remez(f, w, a, b, n, fixed=None, iters=40, grid=1200, tol=1e-7, ref=None,
          want_ref=False):
    """Minimax c_0..c_{n-1} for f on [a, b] with weight w; ``fixed`` maps
    degree -> a value held constant.  Returns (coeffs, max_error), plus the
    final reference set when ``want_ref``; ``ref`` seeds the exchange."""
    fixed = dict(fixed or {})
    m = n - len(fixed)
    a, b = mp.mpf(a), mp.mpf(b)
    if ref is None or len(ref) != m + 1:
        ref = _cheb_points(a, b, m + 1)
    ref = _away_from_weight_zeros(ref, w, a, b)
    best = None
    for _ in range(iters):
        c, E = _solve(f, w, ref, n, fixed)

        def err(z, c=c):
            return w(z) * (f(z) - _poly(c, z))

        pts = _extrema(err, a, b, m + 1, grid)
        emax = max(abs(e) for _, e in pts)
        if best is None or emax < best[1]:
            best = (c, emax, ref)
        if len(pts) < m + 1:
            break
        ref = _away_from_weight_zeros([z for z, _ in pts], w, a, b)
        if abs(E) > 0 and emax / abs(E) - 1 < tol:
            break
    return best if want_ref else best[:2]


def max_error(f, w, a, b, c, grid=3000):
    a, b = mp.mpf(a), mp.mpf(b)
    zs = _cheb_points(a, b, grid)

    def err(z):
        return w(z) * (f(z) - _poly(c, z))

    best = mp.mpf(0)
    es = [err(z) for z in zs]
    for i, z in enumerate(zs):
        if abs(es[i]) > best:
            best = abs(es[i])
            if 0 < i < len(zs) - 1:
                zz, e = _golden_max(err, zs[i - 1], zs[i + 1], 40)
                best = max(best, abs(e))
    return best


def round_to(x, fmt):
    """Nearest value of x in 'f64' or 'f32' (as an mpf)."""
    if fmt == "f64":
        return mp.mpf(float(x))
    if fmt == "f32":
        import numpy as np
        return mp.mpf(float(np.float32(float(x))))
    raise ValueError(fmt)


def remez_rounded(f, w, a, b, n, fmt, fixed=None, pairs=(), iters=40, grid=1200):
    """Greedy rounding: returns (values, max_error) where values[k] is a float
    (or a (hi, lo) pair for k in ``pairs``) and max_error is the true weighted
    error of the rounded polynomial."""
    fixed = dict(fixed or {})
    out = {}
    ref = None
    for k in range(n):
        if k in fixed:
            out[k] = fixed[k]
            continue
        c, _, ref = remez(f, w, a, b, n, fixed=fixed, iters=iters, grid=grid,
                          ref=ref[1:] if ref is not None else None, want_ref=True)
        if k in pairs:
            hi = round_to(c[k], fmt)
            lo = round_to(c[k] - hi, fmt)
            fixed[k] = hi + lo
            out[k] = (float(hi), float(lo))
        else:
            fixed[k] = round_to(c[k], fmt)
            out[k] = float(fixed[k])
    coeffs = [fixed[k] for k in range(n)]
    err = max_error(f, w, a, b, coeffs)
    return [out[k] for k in range(n)], err
