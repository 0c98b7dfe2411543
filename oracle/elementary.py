"""Elementary functions of exact dyadic arguments, as rigorous balls.

Test infrastructure only: nothing in the library path may import this module.

These are textbook definitions chosen to be easy to check by eye and
deliberately different from the methods the GPU kernels use:

* exp:   x = k ln2 + r, exp(r / 2^s) by Taylor series, squared s times.
* log:   x = m 2^E with m in [sqrt(1/2), sqrt 2), log m = 2 atanh((m-1)/(m+1));
         the same series for balls (log_of_ball) and for log(1 + u) with small
         u (log1p_ball, through u / (2 + u)).
* sin/cos: the exact argument times 2/pi (as many bits as its exponent needs),
         nearest integer k and fraction f, r = f pi/2, Taylor series for
         sin r and cos r, quadrant from k mod 4.
* atan:  two argument halvings atan t = 2 atan(t / (1 + sqrt(1 + t^2))), then
         the Taylor series.
* sinh/cosh: Taylor series for |x| < 1, (E -+ 1/E)/2 with E = exp|x| otherwise.
* erf:   (2/sqrt(pi)) e^(-x^2) times the positive series sum 2^n x^(2n+1)/(2n+1)!!.

Every series adds a bound on its truncated tail to the ball radius.
"""
from . import ball as B
from .ball import Ball, exact, add, sub, mul, div, approx, mag_log2
from .consts import pi, ln2, two_over_pi, half_pi

__all__ = ["exp_ball", "log_ball", "log_of_ball", "log1p_ball", "sincos_reduced",
           "sin_cos_ball", "atan_ball", "sinh_cosh_small", "erf_ball", "tail_ball"]


def tail_ball(b, bound_log2):
    """Widen ball b by 2**bound_log2 (a bound on an omitted tail)."""
    if bound_log2 >= b.e:
        sh = bound_log2 - b.e
        return Ball(b.m, b.r + (1 << sh), b.e)
    return Ball(b.m, b.r + 1, b.e)


def _ilog2_floor_upper(b):
    return mag_log2(b)


def exp_ball(x, prec):
    """exp(x) for a ball x with |x| <= 2100 (callers clamp larger args)."""
    if x.m == 0 and x.r == 0:
        return exact(1)
    xa = approx(x)
    k = int(round(xa / 0.6931471805599453))
    wp = prec + 24 + abs(k).bit_length()
    r = sub(x, mul(exact(k), ln2(wp + 8), wp), wp)       # |r| <~ 0.35
    s = 12
    rs = B.scale2(r, -s)                                  # |rs| < 2**-12
    wp2 = prec + 2 * s + 20
    total = exact(1)
    term = exact(1)
    n = 1
    while True:
        term = div(mul(term, rs, wp2), exact(n), wp2)
        total = add(total, term, wp2)
        # the remaining terms are bounded by 2|term| * |rs| < |term| * 2**-11
        if mag_log2(term) < -wp2 - 4:
            total = tail_ball(total, mag_log2(term) - 10)
            break
        n += 1
    for _ in range(s):
        total = mul(total, total, wp2)
    return B.scale2(total, k)


def log_ball(m, e, prec):
    """log(m * 2**e) for an exact positive dyadic (m > 0)."""
    n = m.bit_length()
    E = e + n - 1                         # value = (m / 2**(n-1)) * 2**E
    mant = exact(m, e - E)                # in [1, 2)
    # move the mantissa into [sqrt(1/2), sqrt(2)):  m / 2**(n-1) >= sqrt 2
    # <=> 2 m^2 >= 4**(n-1) * 2 ... compare squares exactly
    if 2 * m * m >= (1 << (2 * (n - 1))) * 4:
        E += 1
        mant = exact(m, e - E)
    wp = prec + 16
    one = exact(1)
    t = div(sub(mant, one, wp), add(mant, one, wp), wp)   # |t| <= 0.1716
    if t.m == 0 and t.r == 0:
        s = exact(0)
    else:
        t2 = mul(t, t, wp)
        term = t
        s = t
        k = 1
        while True:
            term = mul(term, t2, wp)
            s = add(s, div(term, exact(2 * k + 1), wp), wp)
            # tail: sum_{j>k} |t|^(2j+1)/(2j+1) <= |term| * t2 / (1 - t2)
            if mag_log2(term) < mag_log2(t) - wp - 8:
                s = tail_ball(s, mag_log2(term) - 3)
                break
            k += 1
    res = B.scale2(s, 1)
    if E != 0:
        wpe = wp + abs(E).bit_length()
        res = add(res, mul(exact(E), ln2(wpe + 8), wpe), wp)
    return res


def _atanh_series2(t, wp):
    """2 atanh(t) = 2 (t + t^3/3 + t^5/5 + ...) for a ball |t| <= 1/3."""
    if t.m == 0 and t.r == 0:
        return exact(0)
    t2 = mul(t, t, wp)
    term = t
    s = t
    k = 1
    while True:
        term = mul(term, t2, wp)
        s = add(s, div(term, exact(2 * k + 1), wp), wp)
        if mag_log2(term) < mag_log2(t) - wp - 8:
            s = tail_ball(s, mag_log2(term) - 3)
            break
        k += 1
    return B.scale2(s, 1)


def log_of_ball(y, prec):
    """log y for a ball y > 0: y = y' 2^E with the midpoint's exponent, so
    y' is near [1/2, 2); log y' = 2 atanh((y' - 1)/(y' + 1))."""
    lo, hi, e = y.lo_hi()
    if lo <= 0:
        raise B.PrecisionError("log of a ball that reaches zero")
    E = e + y.m.bit_length() - 1
    yp = B.scale2(y, -E)                   # midpoint in [1, 2)
    wp = prec + 16
    one = exact(1)
    res = _atanh_series2(div(sub(yp, one, wp), add(yp, one, wp), wp), wp)
    if E != 0:
        wpe = wp + abs(E).bit_length()
        res = add(res, mul(exact(E), ln2(wpe + 8), wpe), wp)
    return res


def log1p_ball(u, prec):
    """log(1 + u) for a ball u >= 0: 2 atanh(u / (2 + u)) while u < 1 (the
    quotient is below 1/3, and small u keeps its relative accuracy), else
    log(1 + u)."""
    wp = prec + 16
    if approx(u) < 1.0:
        return _atanh_series2(div(u, add(exact(2), u, wp), wp), wp)
    return log_of_ball(add(exact(1), u, wp), prec)


def sincos_reduced(m, e, prec):
    """Reduce the exact x = m * 2**e:  returns (k mod 4, r) with
    x = k * pi/2 + r, |r| <= pi/4 (slightly more in rounding slack), r a ball."""
    if e + m.bit_length() <= -1:          # |x| < 1/2 < pi/4: nothing to do
        return 0, exact(m, e)
    # enough bits of 2/pi that the product's absolute error is < 2**-(prec+64)
    int_bits = max(0, e + m.bit_length())
    wp = prec + int_bits + 96
    y = mul(exact(m, e), two_over_pi(wp), wp)
    # nearest integer to the midpoint (exact integer arithmetic)
    if y.e >= 0:
        k = y.m << y.e
    else:
        k = (y.m + (1 << (-y.e - 1))) >> (-y.e)
    f = sub(y, exact(k), wp)
    r = mul(f, half_pi(prec + 40), prec + 40)
    return k & 3, r


def sin_cos_ball(r, prec):
    """sin r and cos r for a ball |r| <~ 0.8 by Taylor series."""
    wp = prec + 16
    r2 = mul(r, r, wp)
    # sin
    term = r
    s = r
    n = 1
    while True:
        term = div(mul(term, r2, wp), exact((2 * n) * (2 * n + 1)), wp)
        s = add(s, term if n % 2 == 0 else B.neg(term), wp)
        if term.m == 0 or mag_log2(term) < -wp - 8:
            s = tail_ball(s, mag_log2(term) - 2)
            break
        n += 1
    term = exact(1)
    c = exact(1)
    n = 1
    while True:
        term = div(mul(term, r2, wp), exact((2 * n - 1) * (2 * n)), wp)
        c = add(c, term if n % 2 == 0 else B.neg(term), wp)
        if term.m == 0 or mag_log2(term) < -wp - 8:
            c = tail_ball(c, mag_log2(term) - 2)
            break
        n += 1
    return s, c


def atan_ball(t, prec):
    """atan(t) for a ball 0 <= t <= 1."""
    wp = prec + 20
    halvings = 0
    if mag_log2(t) > -20:
        one = exact(1)
        for _ in range(2):
            root = B.sqrt(add(one, mul(t, t, wp), wp), wp)
            t = div(t, add(one, root, wp), wp)
            halvings += 1
    t2 = mul(t, t, wp)
    term = t
    s = t
    k = 1
    while True:
        term = mul(term, t2, wp)
        piece = div(term, exact(2 * k + 1), wp)
        s = add(s, piece if k % 2 == 0 else B.neg(piece), wp)
        if term.m == 0 or mag_log2(term) < mag_log2(t) - wp - 8:
            s = tail_ball(s, mag_log2(term) - 1)
            break
        k += 1
    return B.scale2(s, halvings)


def erf_ball(x, prec):
    """erf x for an exact x > 0: (2/sqrt(pi)) e^(-x^2) sum_n 2^n x^(2n+1) /
    (1 3 5 ... (2n+1)), a series of positive terms (no cancellation).  Once
    the term ratio r = 2x^2/(2n+3) is below 1/2 the tail is below the last
    term."""
    wp = prec + 24
    x2 = mul(x, x, wp)
    twox2 = B.scale2(x2, 1)
    term = x
    s = x
    n = 0
    while True:
        n += 1
        term = div(mul(term, twox2, wp), exact(2 * n + 1), wp)
        s = add(s, term, wp)
        if approx(twox2) < (2 * n + 3) / 2 and mag_log2(term) < mag_log2(s) - wp - 8:
            s = tail_ball(s, mag_log2(term) + 1)
            break
    c = div(exact(2), B.sqrt(pi(wp + 8), wp), wp)
    return mul(mul(c, exp_ball(B.neg(x2), wp), wp), s, wp)


def sinh_cosh_small(x, prec):
    """Taylor series of sinh and cosh for a ball |x| < 1 (no cancellation)."""
    wp = prec + 16
    x2 = mul(x, x, wp)
    term = x
    s = x
    n = 1
    while True:
        term = div(mul(term, x2, wp), exact((2 * n) * (2 * n + 1)), wp)
        s = add(s, term, wp)
        if term.m == 0 or mag_log2(term) < mag_log2(x) - wp - 8:
            s = tail_ball(s, mag_log2(term) - 1)
            break
        n += 1
    term = exact(1)
    c = exact(1)
    n = 1
    while True:
        term = div(mul(term, x2, wp), exact((2 * n - 1) * (2 * n)), wp)
        c = add(c, term, wp)
        if term.m == 0 or mag_log2(term) < -wp - 8:
            c = tail_ball(c, mag_log2(term) - 1)
            break
        n += 1
    return s, c
