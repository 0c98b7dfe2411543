"""Seeded synthetic input generators shared by the tests, the smoke check and
the benchmark.

This module holds no arithmetic of the math functions themselves: it only
draws arguments.  Every array comes from
``np.random.default_rng(SeedSequence([2001, 9258, workload, fn_id, operand]))``
and is generated on the host in the target format.

The paper measures on uniformly distributed arguments in fixed intervals
(Section 7, Table of reciprocal throughputs; the "paper domains" below) and
tests with regular grids, arguments near multiples of pi/2 and random bit
patterns (Section 6).  The five workload mixtures stand in for those; none of
them is a public dataset.

bf16 arrays are returned as float32 arrays holding bf16-representable values
(numpy has no bfloat16); ``to_bf16_bits`` gives the 16-bit patterns.
"""
import numpy as np

__all__ = ["FN_IDS", "rng_for", "specials", "small_set", "mixture", "large_args",
           "narrow_mixture", "batch_requests", "autograd_inputs", "paper_domain",
           "unit_mixture", "function_mixture", "subnormal_results", "SUBNORMAL_FNS",
           "pow_wide", "backward_edges",
           "PAPER_DOMAINS", "round_to_bf16", "to_bf16_bits",
           "from_bf16_bits", "np_dtype"]

FN_IDS = {name: i for i, name in enumerate(
    ["sin", "cos", "tan", "exp", "exp2", "log", "log2", "pow", "atan2",
     "sinh", "cosh", "tanh", "fmod", "remainder", "asin", "acos", "atan",
     "log10", "log1p", "exp10", "expm1", "cbrt", "hypot", "asinh", "acosh", "atanh",
     "erf", "erfc", "fdim", "fmax", "fmin", "sqrt", "trunc", "floor", "ceil", "round",
     "rint", "fabs", "logb", "copysign", "nextafter", "lgamma", "tgamma"])}

DTYPE_MAX = {"f64": np.finfo(np.float64).max, "f32": float(np.finfo(np.float32).max),
             "f16": 65504.0, "bf16": 3.3895313892515355e38}
DTYPE_MIN_SUB = {"f64": 5e-324, "f32": float(np.float32(1.401298464324817e-45)),
                 "f16": 2.0 ** -24, "bf16": 9.183549615799121e-41}


def np_dtype(dt):
    return {"f64": np.float64, "f32": np.float32, "f16": np.float16,
            "bf16": np.float32}[dt]


def rng_for(workload, fn, operand=0):
    fid = FN_IDS[fn] if isinstance(fn, str) else int(fn)
    return np.random.default_rng(np.random.SeedSequence([2001, 9258, workload, fid, operand]))


def round_to_bf16(a):
    """Round float32 values to the nearest bfloat16 (ties to even); NaN stays
    NaN.  Returned as float32."""
    a = np.asarray(a, dtype=np.float32)
    bits = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    out = bits.astype(np.uint32).view(np.float32).copy()
    out[nan] = np.float32("nan")
    return out


def to_bf16_bits(a):
    return (round_to_bf16(a).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b):
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32)


def _cast(x64, dt):
    if dt == "f64":
        return x64.astype(np.float64)
    if dt == "f32":
        return x64.astype(np.float32)
    if dt == "f16":
        return x64.astype(np.float16)
    if dt == "bf16":
        return round_to_bf16(x64.astype(np.float32))
    raise ValueError(dt)


def specials(dt):
    """The special set S of a format: +-0, +-inf, NaN, +-min and +-max
    subnormal."""
    if dt == "f64":
        mins, maxs = 5e-324, float.fromhex("0x0.fffffffffffffp-1022")
    elif dt in ("f32", "bf16"):
        mins = float(np.float32(float.fromhex("0x1p-149")))
        maxs = float(np.float32(float.fromhex("0x1.fffffcp-127")))
        if dt == "bf16":
            mins = float.fromhex("0x1p-133")
            maxs = float.fromhex("0x1.fcp-127")
    else:
        mins, maxs = 2.0 ** -24, float.fromhex("0x1.ff8p-15")
    return np.array([0.0, -0.0, np.inf, -np.inf, np.nan, mins, -mins, maxs, -maxs])


def small_set(fn, n=1 << 20):
    """FP64 sin/cos/exp: U[-10, 10]; log: 1000 * (1 - U[0, 1)) in (0, 1000]."""
    rng = rng_for(1, fn)
    if fn == "log":
        return 1000.0 * (1.0 - rng.random(n))
    return rng.uniform(-10.0, 10.0, n)


def _mixture(rng, n, dt, lo_exp, hi_exp):
    """49% U[-1e4, 1e4], 50% sign * 10^U[lo_exp, hi_exp], 1% uniform over S,
    drawn per element (so waves are mixed)."""
    cat = rng.random(n)
    x = rng.uniform(-1e4, 1e4, n)
    lg_mask = (cat >= 0.49) & (cat < 0.99)
    m = int(lg_mask.sum())
    mag = np.exp(rng.uniform(lo_exp, hi_exp, m) * np.log(10.0))
    sign = np.where(rng.random(m) < 0.5, -1.0, 1.0)
    x[lg_mask] = sign * mag
    sp_mask = cat >= 0.99
    x[sp_mask] = specials(dt)[rng.integers(0, 9, int(sp_mask.sum()))]
    return x


def mixture(fn, dt, n=1 << 26, operand=0):
    rng = rng_for(2, fn, operand)
    if dt == "f64":
        x = _mixture(rng, n, dt, -300.0, 300.0)
    else:
        x = _mixture(rng, n, dt, -38.0, 38.0)
    with np.errstate(over="ignore"):
        return _cast(x, dt)


def large_args(fn, dt, n=1 << 26, operand=0):
    """Large-argument stress.  Trig: half sign * 10^U[5, log10(max)], half
    x = k (pi/2)(1 + delta) with k = floor(10^U[0, 22 - log10(pi/2)]),
    delta ~ U[-1e-3, 1e-3] and delta = 0 for a quarter of those (binary64
    product, so x lies within a few ulps of k pi/2).  fmod/remainder: |x|, |y|
    log-uniform over [min subnormal, max finite], random signs."""
    rng = rng_for(3, fn, operand)
    mx = DTYPE_MAX[dt]
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    if fn in ("fmod", "remainder"):
        lo = np.log10(DTYPE_MIN_SUB[dt])
        hi = np.log10(mx)
        x = sign * 10.0 ** rng.uniform(lo, hi, n)
    else:
        half = rng.random(n) < 0.5
        big = 10.0 ** rng.uniform(5.0, np.log10(mx), n)
        k = np.floor(10.0 ** rng.uniform(0.0, 22.0 - np.log10(np.pi / 2), n))
        delta = rng.uniform(-1e-3, 1e-3, n)
        delta[rng.random(n) < 0.25] = 0.0
        near = k * (np.pi / 2) * (1.0 + delta)
        if dt != "f64":
            near = np.minimum(near, mx)
        x = sign * np.where(half, big, near)
    with np.errstate(over="ignore"):
        return _cast(np.minimum(np.abs(x), mx) * np.sign(x), dt)


def narrow_mixture(fn, dt, n=1 << 28, operand=0):
    """The mixture for bf16/f16 with the log-uniform bounds clamped to
    [min subnormal, max finite] of the format; RNE conversion.  For 'f32' it
    is exactly the binary32 mixture."""
    if dt == "f32":
        return mixture(fn, "f32", n, operand)
    rng = rng_for(4, fn, operand)
    lo = np.log10(DTYPE_MIN_SUB[dt])
    hi = np.log10(DTYPE_MAX[dt])
    lo = max(lo, -38.0)
    hi = min(hi, 38.0)
    x = _mixture(rng, n, dt, lo, hi)
    with np.errstate(over="ignore"):
        return _cast(x, dt)


def unit_mixture(fn, dt, n=1 << 26, operand=0):
    """Arguments for asin/acos, whose domain is [-1, 1]: per element 45%
    U[-1, 1], 25% sign * (1 - 10^U[-16, 0]) (binary32 and narrower: [-7, 0];
    the region next to +-1 where the reduction matters), 20% sign *
    10^U[lo, 0] (tiny arguments down to the format's subnormals), 9% outside
    the domain (sign * 10^U[0, hi], NaN results), 1% the special set."""
    rng = rng_for(8, fn, operand)
    near = -16.0 if dt == "f64" else -7.0
    lo = np.log10(DTYPE_MIN_SUB[dt])
    hi = np.log10(DTYPE_MAX[dt])
    cat = rng.random(n)
    sign = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    x = rng.uniform(-1.0, 1.0, n)
    m = (cat >= 0.45) & (cat < 0.70)
    x[m] = sign[m] * (1.0 - np.exp(rng.uniform(near, 0.0, int(m.sum())) * np.log(10.0)))
    m = (cat >= 0.70) & (cat < 0.90)
    x[m] = sign[m] * np.exp(rng.uniform(lo, 0.0, int(m.sum())) * np.log(10.0))
    m = (cat >= 0.90) & (cat < 0.99)
    x[m] = sign[m] * np.exp(rng.uniform(0.0, hi, int(m.sum())) * np.log(10.0))
    m = cat >= 0.99
    x[m] = specials(dt)[rng.integers(0, 9, int(m.sum()))]
    with np.errstate(over="ignore"):
        return _cast(x, dt)


def function_mixture(fn, dt, n=1 << 26, operand=0):
    """The benchmark-style input of ``fn``: ``unit_mixture`` for asin and
    acos and atanh, otherwise the mixture (bf16/f16: its narrow form); for
    acosh 60% of the elements become |x| + 1 and 30% 1 + 10^U[near, 0].  For log1p a
    fifth of the elements, drawn per element, are -(1 - 10^U[near, 0]) with
    near = -16 (binary64), -7 (binary32, bf16) or -3 (f16): next to -1, where
    1 + x cancels.  For erf and erfc 60% of the elements become U[-w, w]
    (erf) or U[-w, v] (erfc), where w = 6 (binary64) or 4 and v is where erfc
    underflows the format (27.3, 10.1 for binary32 and bf16, 4 for f16): the
    range where the results are neither saturated nor zero.  lgamma and
    tgamma: 40% U[-10, 10], and for tgamma 30% over the range where its
    results are finite and nonzero (binary64 U[-190, 175])."""
    if fn in ("asin", "acos", "atanh"):
        return unit_mixture(fn, dt, n, operand)
    if dt in ("bf16", "f16"):
        x = narrow_mixture(fn, dt, n, operand)
    else:
        x = mixture(fn, dt, n, operand)
    if fn == "log1p":
        rng = rng_for(9, fn, operand)
        m = rng.random(n) < 0.2
        near = {"f64": -16.0, "f16": -3.0}.get(dt, -7.0)
        v = -(1.0 - np.exp(rng.uniform(near, 0.0, int(m.sum())) * np.log(10.0)))
        x[m] = _cast(v, dt)
    if fn == "acosh":
        # the domain is [1, inf): |x| + 1 for 60% of the elements and
        # 1 + 10^U[near, 0] for 30%, the rest as drawn
        rng = rng_for(10, fn, operand)
        c = rng.random(n)
        near = {"f64": -16.0, "f16": -3.0}.get(dt, -7.0)
        with np.errstate(over="ignore"):
            shifted = _cast(np.abs(x.astype(np.float64)) + 1.0, dt)
            close = _cast(1.0 + np.exp(rng.uniform(near, 0.0, n) * np.log(10.0)), dt)
        x = np.where(c < 0.6, shifted, np.where(c < 0.9, close, x))
    if fn in ("lgamma", "tgamma"):
        # 40% U[-10, 10] (both signs, the zeros of lgamma at 1 and 2, the
        # poles), and for tgamma 30% U[-190, 175] (results across the whole
        # range, subnormal ones near -180)
        rng = rng_for(12, fn, operand)
        c = rng.random(n)
        m = c < 0.4
        x[m] = _cast(rng.uniform(-10.0, 10.0, int(m.sum())), dt)
        if fn == "tgamma":
            hi = {"f64": 175.0, "f32": 36.0, "bf16": 36.0, "f16": 9.0}[dt]
            lo = {"f64": -190.0, "f32": -46.0, "bf16": -46.0, "f16": -12.0}[dt]
            m = (c >= 0.4) & (c < 0.7)
            x[m] = _cast(rng.uniform(lo, hi, int(m.sum())), dt)
    if fn in ("erf", "erfc"):
        rng = rng_for(11, fn, operand)
        w = 6.0 if dt == "f64" else 4.0
        v = w if fn == "erf" else {"f64": 27.3, "f16": 4.0}.get(dt, 10.1)
        m = rng.random(n) < 0.6
        x[m] = _cast(rng.uniform(-w, v, int(m.sum())), dt)
    return x


# every (fn, variant) the library serves, used to draw batched requests
REQUEST_KINDS = [("sin", "u10"), ("sin", "u35"), ("cos", "u10"), ("cos", "u35"),
                 ("tan", "u10"), ("tan", "u35"), ("exp", "u10"), ("exp2", "u10"),
                 ("log", "u10"), ("log2", "u10"), ("pow", "u10"), ("atan2", "u10"),
                 ("sinh", "u10"), ("cosh", "u10"), ("tanh", "u10")]


def batch_requests(k=64, lo=3.0, hi=7.0):
    """64 requests: (fn, variant) uniform over the served list, dtype uniform
    over {f64, f32, bf16, f16} (u35 variants only in f64/f32), length
    round(10^U[3, 7])."""
    rng = rng_for(5, 0, 99)
    reqs = []
    for i in range(k):
        fn, var = REQUEST_KINDS[rng.integers(0, len(REQUEST_KINDS))]
        dts = ["f64", "f32"] if var == "u35" else ["f64", "f32", "bf16", "f16"]
        dt = dts[rng.integers(0, len(dts))]
        n = int(round(10.0 ** rng.uniform(lo, hi)))
        reqs.append((fn, var, dt, n, i))
    return reqs


def request_inputs(fn, dt, n, idx):
    a = narrow_mixture(fn, dt, n, operand=1000 + 2 * idx) if dt in ("bf16", "f16") else \
        mixture(fn, dt, n, operand=1000 + 2 * idx)
    b = None
    if fn in ("pow", "atan2"):
        b = narrow_mixture(fn, dt, n, operand=1001 + 2 * idx) if dt in ("bf16", "f16") else \
            mixture(fn, dt, n, operand=1001 + 2 * idx)
    return a, b


def autograd_inputs(fn, n=1 << 24, operand=0):
    rng = rng_for(6, fn, operand)
    return rng.uniform(0.1, 10.0, n).astype(np.float32)


PAPER_DOMAINS = {
    "sin": [(0.4, 0.5), (0.0, 6.28), (0.0, 1e100)],
    "cos": [(0.4, 0.5), (0.0, 6.28), (0.0, 1e100)],
    "tan": [(0.4, 0.5), (0.0, 6.28), (0.0, 1e100)],
    "log": [(0.0, 1e300)],
    "exp": [(-700.0, 700.0)],
    "pow": [(-30.0, 30.0)],
}


def paper_domain(fn, lo, hi, n, dt="f64", operand=0):
    rng = rng_for(7, fn, operand)
    return _cast(rng.uniform(lo, hi, n), dt)


# functions with results in the subnormal range, and how to reach it: an
# argument interval (by format) or "tiny" (subnormal arguments, whose result
# is about the argument itself)
SUBNORMAL_FNS = {
    "exp": {"f64": (-745.2, -708.3), "f32": (-104.0, -87.3)},
    "exp2": {"f64": (-1075.0, -1022.0), "f32": (-150.0, -126.0)},
    "exp10": {"f64": (-323.65, -307.6), "f32": (-45.2, -37.9)},
    "erfc": {"f64": (26.5, 27.3), "f32": (9.1, 10.1)},
    "tgamma": {"f64": (-177.5, -171.5), "f32": (-38.8, -34.3)},
    "pow": "power", "atan2": "quotient", "hypot": "tiny-pair",
    "erf": "tiny", "sin": "tiny", "tan": "tiny", "asin": "tiny", "atan": "tiny",
    "sinh": "tiny", "tanh": "tiny", "asinh": "tiny", "atanh": "tiny",
    "log1p": "tiny", "expm1": "tiny",
}


def subnormal_results(fn, dt, n, operand=0):
    """Arguments (a, b) whose exact results lie in (or at the edge of) the
    subnormal range of binary64 or binary32: uniform over the interval of
    SUBNORMAL_FNS for exp, exp2, exp10 and erfc; random subnormal bit
    patterns of both signs for functions that return about their argument;
    pow: x ~ U(0.01, 0.99), y = t / log2(x) with t ~ U[log2 of the smallest
    subnormal - 1, log2 of the smallest normal], plus exact ties
    (3 2^-215)^5 and the like; atan2: y = x 2^t with x log-uniform; hypot:
    both operands 2^t.  b is None for unary functions."""
    rng = rng_for(8, fn, operand)
    kind = SUBNORMAL_FNS[fn]
    lo_t, hi_t = (-1075.0, -1022.0) if dt == "f64" else (-150.0, -126.0)
    big = 1e300 if dt == "f64" else 1e30
    b = None
    if isinstance(kind, dict):
        lo, hi = kind[dt]
        a = rng.uniform(lo, hi, n)
    elif kind == "tiny":
        nbits = 52 if dt == "f64" else 23
        bits = rng.integers(1, 1 << nbits, n, dtype=np.uint64)
        a = bits.astype(np.float64) * 2.0 ** (lo_t + 1.0)
        a = np.where(rng.random(n) < 0.5, -a, a)
    elif kind == "power":
        a = rng.uniform(0.01, 0.99, n)
        b = rng.uniform(lo_t, hi_t, n) / np.log2(_cast(a, dt).astype(np.float64))
        # exact results halfway between two subnormals, and exact subnormals
        T = -lo_t
        ties = [(3 * 2.0 ** -(T // 5), 5.0), (5 * 2.0 ** -(T // 5), 5.0),
                (2.0 ** -1, T), (2.0, -T), (0.5, T - 1), (9 * 2.0 ** (-(2 * T) // 5), 2.5)]
        for i, (x, y) in enumerate(ties[:n]):
            a[i], b[i] = x, y
    elif kind == "quotient":
        b = np.exp(rng.uniform(0.0, np.log(big), n))
        a = b * 2.0 ** rng.uniform(lo_t, hi_t, n)
        a = np.where(rng.random(n) < 0.5, -a, a)
    else:
        a = 2.0 ** rng.uniform(lo_t + 1.0, hi_t, n)
        b = 2.0 ** rng.uniform(lo_t + 1.0, hi_t, n)
    a = _cast(a, dt)
    return a, None if b is None else _cast(b, dt)


def pow_wide(dt, n, operand=0):
    """pow arguments whose result spans the whole finite range: x log-uniform
    in [1e-3, 1e3], y = w / ln x with w ~ U[-745, 709.7] (binary32:
    U[-103.9, 88.7]), so |y log x| reaches the overflow and underflow edges,
    where the logarithm's relative error is amplified the most."""
    rng = rng_for(9, "pow", operand)
    lo, hi = (-745.0, 709.7) if dt == "f64" else (-103.9, 88.7)
    x = _cast(np.exp(rng.uniform(np.log(1e-3), np.log(1e3), n)), dt)
    y = rng.uniform(lo, hi, n) / np.log(x.astype(np.float64))
    return x, _cast(y, dt)


def backward_edges(fn, dt, n, operand=0):
    """Arguments for the backward kernels away from U[0.1, 10]:
    pow: the pow_wide range (partials near overflow and underflow) with
    negative x at integer y mixed in; atan2: y, x both log-uniform over
    1e-300..1e300 (binary32: 1e-37..1e37) with random signs and a ratio
    within e^+-3; tanh: x ~ U[-380, 380] (binary32: U[-60, 60]); tan: doubles
    next to odd multiples of pi/2 come from the tests' own hard-case list.
    Returns (a, b, g) with g standard normal; b is None for unary functions."""
    rng = rng_for(10, fn, operand)
    g = _cast(rng.standard_normal(n), dt)
    b = None
    if fn == "pow":
        a, b = pow_wide(dt, n, operand)
        neg = rng.random(n) < 0.25
        yi = np.rint(rng.uniform(-40.0, 40.0, n))
        a = np.where(neg, -a.astype(np.float64), a.astype(np.float64))
        b = np.where(neg, yi, b.astype(np.float64))
        a, b = _cast(a, dt), _cast(b, dt)
    elif fn == "atan2":
        e = 300.0 if dt == "f64" else 37.0
        a = np.exp(rng.uniform(-e, e, n) * np.log(10.0))
        b = a * np.exp(rng.uniform(-3.0, 3.0, n))
        a = np.where(rng.random(n) < 0.5, -a, a)
        b = np.where(rng.random(n) < 0.5, -b, b)
        a, b = _cast(a, dt), _cast(b, dt)
    elif fn == "tanh":
        m = 380.0 if dt == "f64" else 60.0
        a = _cast(rng.uniform(-m, m, n), dt)
    else:
        raise ValueError(fn)
    return a, b, g
