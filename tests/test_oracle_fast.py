"""Pins of the oracle's fast binary32 stage (oracle/fast/fast32.c) for sin,
cos, tan, exp, exp2, log, log2, sinh, cosh and tanh, independently of its
own arithmetic:

* against mpmath at 300 bits: the double-double value within the claimed
  2^-90 relative (random bit patterns, each function's domain, arguments
  next to multiples of pi/2, exp near its overflow and underflow limits, log
  next to 1);
* against the ball oracle: the same correctly rounded binary32 result
  (undecided inputs go to the ball oracle by construction);
* the sweep against the host libm's binary64 results rounded to binary32
  over 2^18-pattern stretches: every difference is a double rounding, and
  the ball oracle sides with the fast stage on each;
* the ULP check against known answers (the oracle's own results, results
  one ulp away, a NaN where a number is due).
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from oracle import fast32

MPF = {"sin": mp.sin, "cos": mp.cos, "tan": mp.tan, "exp": mp.exp, "exp2": lambda v: mp.mpf(2) ** v,
       "log": mp.log, "log2": lambda v: mp.log(v, 2), "sinh": mp.sinh, "cosh": mp.cosh,
       "tanh": mp.tanh}
FNS = list(MPF)


@pytest.fixture(scope="module", autouse=True)
def _built():
    fast32.load()                       # builds the C stage if it is missing


def _inputs(fn, n=1200, seed=3):
    rng = np.random.default_rng(seed + len(fn))
    bits = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    parts = [bits.view(np.float32)]
    if fn in ("sin", "cos", "tan"):
        k = np.concatenate([np.arange(1, 400), rng.integers(1, 1 << 40, 300)]).astype(np.float64)
        near = (k * (math.pi / 2)).astype(np.float32)
        parts += [near, np.nextafter(near, np.float32(0)), rng.uniform(-10, 10, 300).astype(np.float32),
                  np.float32([7.729179e28, 21999384576.0, 1.5458358e29, 1e-40, 3.4028235e38])]
    elif fn == "exp":
        parts += [rng.uniform(-104, 89, 600).astype(np.float32),
                  np.float32([88.72283, 88.72284, -103.97208, -103.9721, -87.33655, 1e-30, -1e-30])]
    elif fn == "exp2":
        parts += [rng.uniform(-151, 129, 600).astype(np.float32),
                  np.float32([127.99999, 128.0, -149.0, -149.5, -150.0, 0.5, 1e-30])]
    elif fn in ("sinh", "cosh", "tanh"):
        parts += [rng.uniform(-95, 95, 400).astype(np.float32),
                  (np.exp(rng.uniform(-60, 0, 200)) * rng.choice([-1, 1], 200)).astype(np.float32),
                  np.float32([0.0625, -0.0624999, 89.4, 89.5, 20.0, 9.0, 1e-40])]
    else:
        parts += [np.exp(rng.uniform(-100, 88, 600)).astype(np.float32),
                  (1 + rng.uniform(-1e-3, 1e-3, 200)).astype(np.float32),
                  np.float32([1.0, 0.99999994, 1.0000001, 1e-45, 3.4028235e38])]
    return np.concatenate(parts).astype(np.float32)


@pytest.mark.parametrize("fn", FNS)
def test_pair_within_claimed_bound_of_mpmath(fn):
    x = _inputs(fn, n=300)
    rn, hi, lo, und = fast32.fast_eval(fn, x)
    mp.mp.prec = 300
    worst = mp.mpf(0)
    for xi, h, l in zip(x, hi, lo):
        if not (np.isfinite(h) and np.isfinite(xi)) or h == 0:
            continue
        if fn in ("log", "log2") and xi <= 0:
            continue
        exact = MPF[fn](mp.mpf(float(xi)))
        if exact == 0 or abs(exact) > mp.mpf(2) ** 128 or abs(exact) < mp.mpf(2) ** -150:
            continue
        rel = abs((mp.mpf(float(h)) + mp.mpf(float(l))) - exact) / abs(exact)
        worst = max(worst, rel)
    assert worst <= mp.mpf(2) ** -90, (fn, float(mp.log(worst, 2)))


@pytest.mark.parametrize("fn", FNS)
def test_rounded_results_match_the_ball_oracle(fn):
    x = _inputs(fn)
    rn, hi, lo = fast32.evaluate(fn, x)
    rb = oracle.evaluate(fn, "f32", x.astype(np.float64))[0]
    same = (rn == rb) | (np.isnan(rn) & np.isnan(rb))
    same &= (np.signbit(rn) == np.signbit(rb)) | np.isnan(rb)
    assert same.all(), x[~same][:5]


@pytest.mark.parametrize("fn,start", [("sin", 0x3f800000), ("sin", 0x4e000000),
                                      ("cos", 0x40490000), ("tan", 0x3fc90000),
                                      ("exp", 0x42000000), ("exp", 0xc2c00000),
                                      ("exp2", 0xc3100000), ("log", 0x3f7f0000),
                                      ("log", 0x00000001), ("log2", 0x3f800000),
                                      ("sinh", 0x3d800000), ("cosh", 0x42b00000),
                                      ("tanh", 0x3c000000)])
def test_sweep_against_libm_double_rounded(fn, start):
    st, differ, und = fast32.sweep_libm(fn, start, 1 << 18)
    assert st.n == 1 << 18
    assert st.differ == st.differ_explained, (st.differ, st.differ_explained)
    # the ball oracle sides with the fast stage wherever they differ from libm
    if differ.size:
        x = differ[:64].view(np.float32)
        rb = oracle.evaluate(fn, "f32", x.astype(np.float64))[0]
        rf = fast32.fast_eval(fn, x)[0]
        assert np.array_equal(rb, rf.astype(np.float64))
    assert st.undecided == und.size


def test_check_metric_on_known_answers():
    start, n = 0x3f000000, 1 << 14
    x = np.arange(start, start + n, dtype=np.uint64).astype(np.uint32).view(np.float32)
    rn = fast32.evaluate("exp", x)[0].astype(np.float32)
    st, bad, _ = fast32.check("exp", start, n, rn, 1.0)
    assert st.violations == 0 and st.special_mismatch == 0 and st.max_ulp <= 0.5
    up = np.nextafter(rn, np.float32(np.inf))
    st, bad, _ = fast32.check("exp", start, n, up, 1.0)
    assert 0.5 < st.max_ulp < 1.5
    st, bad, _ = fast32.check("exp", start, n, up, 0.75)
    assert st.violations > 0
    y = rn.copy()
    y[5] = np.nan
    st, bad, _ = fast32.check("exp", start, n, y, 1.0)
    assert st.violations == 1 and bad[0] == start + 5


# ---- the binary64 stage (oracle/fast/fast64.c) -------------------------------

from oracle import fast64  # noqa: E402
import workloads as W  # noqa: E402


def _inputs64(fn, n=800, seed=4):
    rng = np.random.default_rng(seed + len(fn))
    parts = [W.mixture(fn, "f64", n, 7), rng.integers(0, 1 << 63, n // 2, dtype=np.uint64).view(np.float64),
             -rng.integers(0, 1 << 63, n // 4, dtype=np.uint64).view(np.float64)]
    if fn in ("sin", "cos", "tan"):
        k = rng.integers(1, 1 << 50, 200).astype(np.float64)
        near = k * (math.pi / 2)
        parts += [near, np.nextafter(near, 0.0),
                  np.array([6381956970095103 * 2.0 ** 797, 5988794123081509 * 2.0 ** 816, 1e22,
                            2.0 ** 1023, 0.7853981633974483, 5e-324])]
    elif fn in ("exp", "exp2"):
        lo, hi = (-746.0, 710.0) if fn == "exp" else (-1076.0, 1025.0)
        parts += [rng.uniform(lo, hi, 400), np.array([709.78, 709.79, -745.13, -708.4, -1074.5, 1023.9])]
    elif fn in ("sinh", "cosh", "tanh"):
        parts += [rng.uniform(-715, 715, 300), np.exp(rng.uniform(-700, 0, 200)),
                  np.array([0.0625, 40.0, 40.1, 710.4, 710.5, 1e-310])]
    else:
        parts += [np.exp(rng.uniform(-740, 709, 400)), 1 + rng.uniform(-1e-9, 1e-9, 100),
                  np.array([1.0, 0.9999999999999999, 5e-324, 1.7976931348623157e308])]
    return np.concatenate(parts)


@pytest.mark.parametrize("fn", FNS)
def test_fast64_pair_within_claimed_bound_of_mpmath(fn):
    x = _inputs64(fn, n=150)
    rn, hi, lo, und = fast64.fast_eval(fn, x)
    mp.mp.prec = 300
    worst = mp.mpf(0)
    for xi, h, l in zip(x, hi, lo):
        if not (np.isfinite(h) and np.isfinite(xi)) or h == 0:
            continue
        if fn in ("log", "log2") and xi <= 0:
            continue
        exact = MPF[fn](mp.mpf(float(xi)))
        # the pair is returned scaled: below 2^-960 its low word loses bits
        if exact == 0 or abs(exact) > mp.mpf(2) ** 1023 or abs(exact) < mp.mpf(2) ** -960:
            continue
        worst = max(worst, abs((mp.mpf(float(h)) + mp.mpf(float(l))) - exact) / abs(exact))
    assert worst <= mp.mpf(2) ** -90, (fn, float(mp.log(worst, 2)))


@pytest.mark.parametrize("fn", FNS)
def test_fast64_rounded_results_match_the_ball_oracle(fn):
    x = _inputs64(fn)
    rn, hi, lo = fast64.evaluate(fn, x)
    rb = oracle.evaluate(fn, "f64", x)[0]
    same = (rn == rb) | (np.isnan(rn) & np.isnan(rb))
    same &= (np.signbit(rn) == np.signbit(rb)) | np.isnan(rb)
    assert same.all(), x[~same][:5]


def test_fast64_check_metric_on_known_answers():
    x = W.mixture("exp", "f64", 1 << 14, 3)
    rn = fast64.evaluate("exp", x)[0]
    tot = fast64.check_all("exp", x, rn, 1.0, threads=2, chunk=1 << 12)
    assert tot["violations"] == 0 and tot["special_mismatch"] == 0 and tot["max_ulp"] <= 0.5
    finite = np.isfinite(rn) & (np.abs(rn) >= 2.0 ** -1022)
    # one ulp up, away from powers of two (where the binade below has half the ulp)
    finite &= np.frexp(rn)[0] != 0.5
    up = np.where(finite, np.nextafter(rn, np.inf), rn)
    tot = fast64.check_all("exp", x, up, 1.0, threads=2, chunk=1 << 12)
    assert 0.5 < tot["max_ulp"] < 1.5 and tot["special_mismatch"] == 0
    y = rn.copy()
    i = int(np.nonzero(finite)[0][3])
    y[i] = np.nan
    tot = fast64.check_all("exp", x, y, 1.0, threads=2, chunk=1 << 12)
    assert tot["violations"] == 1 and tot["bad"][0] == i


# ---- pow and atan2 in the binary64 stage (oracle/fast/binary.h) ------------

BIN_BOUND = {"pow": 2.0 ** -86, "atan2": 2.0 ** -90}


def _inputs64_2(fn, n=600, seed=9):
    rng = np.random.default_rng(seed + len(fn))
    sp = W.specials("f64")
    a = [W.mixture(fn, "f64", n, 11), np.repeat(sp, sp.size)]
    b = [W.mixture(fn, "f64", n, 12), np.tile(sp, sp.size)]
    if fn == "pow":
        x = 1.0 + rng.uniform(-1e-6, 1e-6, 150)                  # near 1, large exponents
        a += [x, np.exp(rng.uniform(-5, 5, 300))]
        w = rng.uniform(-746.0, 710.0, 300)                       # every result range, subnormals too
        b += [rng.uniform(-1e8, 1e8, 150), w / np.log(a[-1])]
        m = rng.integers(1, 40, 150).astype(np.float64)           # exact results and negative bases
        k = rng.integers(-30, 30, 150).astype(np.float64)
        a += [m, -m, np.full(40, -1.0), 2.0 ** rng.integers(-1074, 1023, 40).astype(np.float64)]
        b += [k, k, rng.integers(-2 ** 60, 2 ** 60, 40).astype(np.float64),
              rng.uniform(-3, 3, 40)]
    else:
        y = rng.standard_normal(300) * 10.0 ** rng.uniform(-300, 300, 300)
        x = rng.standard_normal(300) * 10.0 ** rng.uniform(-300, 300, 300)
        near = y * (1 + rng.uniform(-1e-12, 1e-12, 300))          # |y| close to |x|
        sub = rng.integers(1, 1 << 40, 100).astype(np.float64) * 5e-324
        a += [y, near, sub, -sub, np.full(100, 1e-300)]
        b += [x, y * np.sign(rng.standard_normal(300)), rng.uniform(1, 1e5, 100),
              -rng.uniform(1, 1e5, 100), rng.uniform(1e10, 1e300, 100)]
    return np.concatenate(a), np.concatenate(b)


def _mp2(fn, a, b):
    if fn == "atan2":
        return mp.atan2(mp.mpf(float(a)), mp.mpf(float(b)))
    return mp.power(mp.mpf(float(a)), mp.mpf(float(b)))


@pytest.mark.parametrize("fn", ["pow", "atan2"])
def test_fast64_binary_pair_within_claimed_bound_of_mpmath(fn):
    a, b = _inputs64_2(fn, n=100)
    rn, hi, lo, und = fast64.fast_eval(fn, a, b)
    mp.mp.prec = 300
    worst = mp.mpf(0)
    checked = 0
    for ai, bi, h, l, r in zip(a, b, hi, lo, rn):
        if not (np.isfinite(h) and np.isfinite(r)) or h == 0 or r == 0 or ai == 0 or bi == 0:
            continue                                              # signed zeros: see the next test
        exact = _mp2(fn, ai, bi)
        if exact == 0 or abs(exact) > mp.mpf(2) ** 1023 or abs(exact) < mp.mpf(2) ** -960:
            continue
        if l == 0 and mp.mpf(float(h)) == exact:
            continue                                              # exact special value
        worst = max(worst, abs((mp.mpf(float(h)) + mp.mpf(float(l))) - exact) / abs(exact))
        checked += 1
    assert checked > 500
    assert worst <= BIN_BOUND[fn], (fn, float(mp.log(worst, 2)))


@pytest.mark.parametrize("fn", ["pow", "atan2"])
def test_fast64_binary_rounded_results_match_the_ball_oracle(fn):
    a, b = _inputs64_2(fn)
    rn, hi, lo = fast64.evaluate(fn, a, b)
    rb = oracle.evaluate(fn, "f64", a, b)[0]
    same = (rn == rb) | (np.isnan(rn) & np.isnan(rb))
    same &= (np.signbit(rn) == np.signbit(rb)) | np.isnan(rb)
    assert same.all(), (a[~same][:5], b[~same][:5], rn[~same][:5], rb[~same][:5])


def _inputs32_2(fn, n=3000, seed=21):
    rng = np.random.default_rng(seed + len(fn))
    sp = W.specials("f32")
    a = [W.mixture(fn, "f32", n, 13), np.repeat(sp, sp.size)]
    b = [W.mixture(fn, "f32", n, 14), np.tile(sp, sp.size)]
    if fn == "pow":
        x = np.exp(rng.uniform(-5, 5, 1000)).astype(np.float32)
        w = rng.uniform(-104.0, 89.0, 1000)                       # every result range, subnormals too
        a += [x, rng.integers(1, 40, 300).astype(np.float32)]
        b += [(w / np.log(x.astype(np.float64))).astype(np.float32),
              rng.integers(-30, 30, 300).astype(np.float32)]
        a += [-a[-1]]
        b += [b[-1]]
    else:
        a += [(rng.standard_normal(1000) * 10.0 ** rng.uniform(-38, 38, 1000)).astype(np.float32),
              (rng.integers(1, 1 << 20, 300) * 2.0 ** -149).astype(np.float32)]
        b += [(rng.standard_normal(1000) * 10.0 ** rng.uniform(-38, 38, 1000)).astype(np.float32),
              rng.uniform(1, 1e5, 300).astype(np.float32)]
    return np.concatenate(a).astype(np.float32), np.concatenate(b).astype(np.float32)


@pytest.mark.parametrize("fn", ["pow", "atan2"])
def test_fast32_binary_rounded_results_match_the_ball_oracle(fn):
    a, b = _inputs32_2(fn)
    rn = fast32.evaluate(fn, a, b)[0]
    rb = oracle.evaluate(fn, "f32", a.astype(np.float64), b.astype(np.float64))[0]
    same = (rn == rb) | (np.isnan(rn) & np.isnan(rb))
    same &= (np.signbit(rn) == np.signbit(rb)) | np.isnan(rb)
    assert same.all(), (a[~same][:5], b[~same][:5], rn[~same][:5], rb[~same][:5])


@pytest.mark.parametrize("fn", ["pow", "atan2"])
def test_binary_check_metric_on_known_answers(fn):
    """check_all over correctly rounded results, one ulp off, and a NaN."""
    for dt, fast in (("f64", fast64), ("f32", fast32)):
        a = W.mixture(fn, dt, 1 << 13, 31)
        b = W.mixture(fn, dt, 1 << 13, 32)
        rn = fast.evaluate(fn, a, b)[0].astype(a.dtype)
        tot = fast.check_all(fn, a, rn, 1.0, threads=2, chunk=1 << 11, z=b)
        assert tot["violations"] == 0 and tot["special_mismatch"] == 0 and tot["max_ulp"] <= 0.5
        tiny = 2.0 ** (-1022 if dt == "f64" else -126)
        ok = np.isfinite(rn) & (np.abs(rn) >= tiny) & (np.frexp(rn)[0] != 0.5)
        up = np.where(ok, np.nextafter(rn, np.asarray(np.inf, rn.dtype)), rn)
        tot = fast.check_all(fn, a, up, 1.0, threads=2, chunk=1 << 11, z=b)
        assert 0.5 < tot["max_ulp"] < 1.5 and tot["special_mismatch"] == 0, (dt, tot["max_ulp"])
        y = rn.copy()
        i = int(np.nonzero(ok)[0][5])
        y[i] = np.nan
        tot = fast.check_all(fn, a, y, 1.0, threads=2, chunk=1 << 11, z=b)
        assert tot["violations"] == 1 and tot["bad"][0] == i


# ---- asin, acos, atan, log10, log1p, exp10, expm1, cbrt in both stages -------
# (oracle/fast/binary.h)

INV = {"asin": mp.asin, "acos": mp.acos, "atan": mp.atan, "log10": mp.log10, "log1p": mp.log1p,
       "exp10": lambda v: mp.mpf(10) ** v, "expm1": mp.expm1,
       "cbrt": lambda v: mp.sign(v) * mp.cbrt(abs(v)), "asinh": mp.asinh, "acosh": mp.acosh,
       "atanh": mp.atanh, "erf": mp.erf, "erfc": mp.erfc}


def _inputs_inv(fn, dt, n=400, seed=41):
    rng = np.random.default_rng(seed + len(fn) + len(dt))
    npdt = np.float64 if dt == "f64" else np.float32
    near1 = 1 - 10.0 ** -rng.uniform(0, 15 if dt == "f64" else 7, n // 4)
    parts = [W.function_mixture(fn, dt, n, 43), W.specials(dt), rng.uniform(-1, 1, n),
             near1, -near1, 10.0 ** -rng.uniform(0, 300 if dt == "f64" else 44, n // 4),
             np.array([1.0, -1.0, 0.5, -0.5, 2.0 ** -30, 2.0 ** -31, 0.9999999])]
    wide = np.sign(rng.standard_normal(n)) * 10.0 ** rng.uniform(-300 if dt == "f64" else -44,
                                                                  300 if dt == "f64" else 38, n)
    if fn in ("atan", "cbrt", "log10", "log1p"):
        parts += [wide, np.abs(wide), 10.0 ** rng.integers(0, 22, 40), (np.arange(1, 60) ** 3)]
    if fn in ("exp10", "expm1"):
        lim = (310, 330) if dt == "f64" else (39, 46)
        parts += [rng.uniform(-lim[1], lim[0], n), rng.uniform(-0.5, 0.5, n), wide[:n // 4],
                  np.arange(-20, 23, dtype=np.float64)]
    if fn == "expm1":
        lim = 712 if dt == "f64" else 90
        parts += [rng.uniform(-lim, lim, n), np.array([0.3, -0.3, 0.29999, 709.7, 88.7, -40.0])]
    if fn == "log1p":
        parts += [rng.uniform(-1, 0, n), -1 + 10.0 ** -rng.uniform(0, 15, n // 4)]
    if fn in ("asinh", "acosh"):
        parts += [wide, np.abs(wide), rng.uniform(-3, 3, n), 1 + 10.0 ** -rng.uniform(0, 15, n // 4),
                  np.array([0.4, 0.39999, 1.0, 2.0 ** 500, 2.0 ** 501, 1e300])]
    if fn == "atanh":
        parts += [np.array([0.171, 0.17100001, -0.171, 0.5, -0.99999])]
    if fn in ("erf", "erfc"):
        top = 28 if dt == "f64" else 10.5
        parts += [rng.uniform(-7, top, n), rng.uniform(1.9, 2.1, n // 4), rng.uniform(5.5, 6.5, n // 4),
                  np.array([2.0, -2.0, 6.0, -6.0, 26.55, 27.2, 9.19, 10.05])]
    return np.concatenate(parts).astype(npdt)


@pytest.mark.parametrize("fn", list(INV))
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_c99_pair_within_claimed_bound_of_mpmath(fn, dt):
    fast = fast64 if dt == "f64" else fast32
    x = _inputs_inv(fn, dt, n=150)
    rn, hi, lo, und = fast.fast_eval(fn, x)
    mp.mp.prec = 300
    worst = mp.mpf(0)
    checked = 0
    for xi, h, l in zip(x, hi, lo):
        if not (np.isfinite(h) and np.isfinite(xi)) or h == 0:
            continue
        exact = INV[fn](mp.mpf(float(xi)))
        if exact == 0 or abs(exact) < mp.mpf(2) ** -960 or abs(exact) > mp.mpf(2) ** 1023:
            continue
        if l == 0 and mp.mpf(float(h)) == exact:
            continue                                              # an exact value
        worst = max(worst, abs((mp.mpf(float(h)) + mp.mpf(float(l))) - exact) / abs(exact))
        checked += 1
    assert checked > 200
    assert worst <= mp.mpf(2) ** -90, (fn, dt, float(mp.log(worst, 2)))


@pytest.mark.parametrize("fn", list(INV))
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_c99_rounded_results_match_the_ball_oracle(fn, dt):
    fast = fast64 if dt == "f64" else fast32
    x = _inputs_inv(fn, dt)
    rn = fast.evaluate(fn, x)[0].astype(np.float64)
    rb = oracle.evaluate(fn, dt, x.astype(np.float64))[0]
    same = (rn == rb) | (np.isnan(rn) & np.isnan(rb))
    same &= (np.signbit(rn) == np.signbit(rb)) | np.isnan(rb)
    assert same.all(), (x[~same][:5], rn[~same][:5], rb[~same][:5])


@pytest.mark.parametrize("fn,start", [("asin", 0x3f000000), ("asin", 0x3f7f0000),
                                      ("acos", 0x3e800000), ("acos", 0xbf7f0000),
                                      ("atan", 0x3f700000), ("atan", 0x4b000000),
                                      ("log10", 0x3f7f0000), ("log10", 0x41200000),
                                      ("log1p", 0x38000000), ("log1p", 0xbf000000),
                                      ("exp10", 0x3f000000), ("exp10", 0xc2100000),
                                      ("expm1", 0x3e800000), ("expm1", 0xbe900000),
                                      ("cbrt", 0x3f800000), ("cbrt", 0x00400000),
                                      ("asinh", 0x3e000000), ("asinh", 0x4f000000),
                                      ("acosh", 0x3f800000), ("acosh", 0x40000000),
                                      ("atanh", 0x3e200000), ("atanh", 0xbf700000),
                                      ("erf", 0x3f800000), ("erf", 0xc0000000),
                                      ("erfc", 0x40000000), ("erfc", 0x41100000)])
def test_c99_sweep_against_libm_double_rounded(fn, start):
    st, differ, und = fast32.sweep_libm(fn, start, 1 << 18)
    assert st.n == 1 << 18
    assert st.differ == st.differ_explained, (st.differ, st.differ_explained)
    if differ.size:
        x = differ[:64].view(np.float32)
        rb = oracle.evaluate(fn, "f32", x.astype(np.float64))[0]
        rf = fast32.fast_eval(fn, x)[0]
        assert np.array_equal(rb, rf.astype(np.float64))
    assert st.undecided == und.size


# ---- lgamma and tgamma in both stages (oracle/fast/binary.h) ------------------

def _gamma_exact(fn, v):
    v = mp.mpf(v)
    if fn == "lgamma":
        return mp.loggamma(v) if v > 0 else mp.log(abs(mp.gamma(v)))
    return mp.gamma(v)


def _inputs_gamma(fn, dt="f32", n=400, seed=47):
    rng = np.random.default_rng(seed + len(fn) + len(dt))
    zeros = np.array([1.0, 2.0, -2.4570247, -2.7476826, -3.1435917, -3.9552288, -4.0390536,
                      -4.9991650, -5.0008322])
    near = (zeros[:, None] * (1 + rng.uniform(-2e-6, 2e-6, (zeros.size, n // 20)))).ravel()
    tiny, big = (44, 38) if dt == "f32" else (320, 308)
    parts = [W.function_mixture(fn, dt, n, 43), W.specials(dt), rng.uniform(0, 40, n),
             rng.uniform(-45, 0, n), near, 10.0 ** -rng.uniform(0, tiny, n // 4),
             -(10.0 ** -rng.uniform(0, tiny, n // 4)), 10.0 ** rng.uniform(0, big, n // 4),
             np.arange(-50, 60) + rng.uniform(-1e-5, 1e-5, 110), np.arange(-5.0, 40.0),
             np.array([0.5, -0.5, 1.5, -1.5, 34.0, 35.04, 35.05, -38.0001, -41.99, 19.9999, 20.0,
                       2.0 ** -127, 2.0 ** -128, -(2.0 ** -128), 4e36, 4.1e36])]
    if dt == "f64":
        parts += [rng.uniform(-190, 180, n), -(10.0 ** rng.uniform(0, 15.6, n // 4)),
                  np.array([171.6, 171.7, -184.1, -190.5, 2.0 ** 1000, 2.0 ** 1001, 2.5e305,
                            2.6e305, 1.7e308, 5e-324, -5e-324, 2.0 ** -500, -(2.0 ** -500),
                            1 - 2.0 ** -40, 2 + 2.0 ** -40, -(2.0 ** 52) + 0.5])]
    return np.concatenate(parts).astype(np.float64 if dt == "f64" else np.float32)


@pytest.mark.parametrize("fn", ["lgamma", "tgamma"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_gamma_pair_within_its_claimed_bound_of_mpmath(fn, dt):
    fast = fast64 if dt == "f64" else fast32
    x = _inputs_gamma(fn, dt, n=200)
    rn, hi, lo, und = fast.fast_eval(fn, x)
    rel = fast.fast_rel(fn, x)
    mp.mp.prec = 300
    checked = 0
    for xi, h, l, r in zip(x, hi, lo, rel):
        if not (np.isfinite(h) and np.isfinite(xi)) or r == 0.0:
            continue
        exact = _gamma_exact(fn, float(xi))
        if abs(exact) > mp.mpf(2) ** 1023 or abs(exact) < mp.mpf(2) ** -960:
            continue                                   # the pair is scaled there
        err = abs((mp.mpf(float(h)) + mp.mpf(float(l))) - exact) / abs(exact)
        assert err <= r, (fn, float(xi), float(mp.log(err, 2)), np.log2(r))
        checked += 1
    assert checked > 300
    # the bound is typically 2^-88 or tighter away from the zeros of log Gamma
    far = np.isfinite(x) & (np.abs(x - np.round(np.nan_to_num(x))) > 0.1)
    assert np.median(rel[far & (rel > 0)]) < 2.0 ** -88


@pytest.mark.parametrize("fn", ["lgamma", "tgamma"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_gamma_rounded_results_match_the_ball_oracle(fn, dt):
    fast = fast64 if dt == "f64" else fast32
    x = _inputs_gamma(fn, dt)
    rn = fast.evaluate(fn, x)[0].astype(np.float64)
    rb = oracle.evaluate(fn, dt, x.astype(np.float64))[0]
    same = (rn == rb) | (np.isnan(rn) & np.isnan(rb))
    same &= (np.signbit(rn) == np.signbit(rb)) | np.isnan(rb)
    assert same.all(), (x[~same][:5], rn[~same][:5], rb[~same][:5])


def test_gamma_known_values():
    """Closed forms: Gamma(n) = (n - 1)!, Gamma(1/2) = sqrt(pi),
    Gamma(-1/2) = -2 sqrt(pi), log Gamma(3/2) = log(sqrt(pi)/2), the C99
    special values, and the sign of Gamma on the negative intervals."""
    n = np.arange(1, 35, dtype=np.float32)
    fact = np.array([float(mp.factorial(k - 1)) for k in range(1, 35)])
    assert np.array_equal(fast32.fast_eval("tgamma", n)[0], fact.astype(np.float32))
    sp = np.float32(mp.sqrt(mp.pi))
    x = np.array([0.5, -0.5], np.float32)
    assert list(fast32.fast_eval("tgamma", x)[0]) == [sp, np.float32(-2 * mp.sqrt(mp.pi))]
    assert fast32.fast_eval("lgamma", np.array([1.5], np.float32))[0][0] == \
        np.float32(mp.log(mp.sqrt(mp.pi) / 2))
    sv = np.array([0.0, -0.0, 1.0, 2.0, -1.0, -7.0, np.inf, -np.inf, np.nan], np.float32)
    lg = fast32.fast_eval("lgamma", sv)[0]
    assert np.array_equal(lg[:2], [np.inf, np.inf]) and lg[2] == 0 and lg[3] == 0
    assert not np.signbit(lg[2]) and not np.signbit(lg[3])
    assert np.all(lg[4:8] == np.inf) and np.isnan(lg[8])
    tg = fast32.fast_eval("tgamma", sv)[0]
    assert tg[0] == np.inf and tg[1] == -np.inf and tg[2] == 1 and tg[3] == 1
    assert np.isnan(tg[4]) and np.isnan(tg[5]) and tg[6] == np.inf and np.isnan(tg[7])
    mids = -np.arange(0, 30) - np.float32(0.5)
    sg = np.sign(fast32.fast_eval("tgamma", mids.astype(np.float32))[0])
    assert np.array_equal(sg[:20], [(-1.0) ** (k + 1) for k in range(20)])


@pytest.mark.parametrize("fn,start", [("lgamma", 0x40400000), ("lgamma", 0x41a00000),
                                      ("lgamma", 0xc0b00000), ("tgamma", 0x3f000000),
                                      ("tgamma", 0x41000000), ("tgamma", 0xc1200000)])
def test_gamma_sweep_against_libm_double_rounded(fn, start):
    st, differ, und = fast32.sweep_libm(fn, start, 1 << 17)
    assert st.n == 1 << 17
    assert st.differ == st.differ_explained, (st.differ, st.differ_explained)
    if differ.size:
        x = differ[:64].view(np.float32)
        rb = oracle.evaluate(fn, "f32", x.astype(np.float64))[0]
        rf = fast32.fast_eval(fn, x)[0]
        assert np.array_equal(rb, rf.astype(np.float64))
    assert st.undecided == und.size
