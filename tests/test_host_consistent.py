"""The host build of the bit-consistent evaluators (libm_hip_host.so) meets
the same bounds as the GPU entry points against the oracle: 1.0 ULP (u10),
3.5 ULP (u35), exact fmod/remainder, Annex F special values bit-exact.  It
runs on the CPU; the GPU half of the bit-identity check is
test_gpu_consistent.py.  This also pins the bit-consistent primitives
(IEEE division and square root in place of the hardware estimates, the
FMA-only x^(-1/3) seed of cbrt)."""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.ulp import compare, exact_compare

import paper_2001_09258_amd as L

N = 3000
KINDS = [(fn, v, dt) for fn in L.UNARY + L.BINARY for v in L.VARIANTS[fn]
         for dt in ("f64", "f32")]
BOUND = {"u10": 1.0, "u35": 3.5, "exact": 0.0}


def _inputs(fn, dt, operand):
    a = W.function_mixture(fn, dt, N, 500 + operand)
    sp = W.specials(dt)
    a[:sp.size] = sp
    return a


@pytest.fixture(scope="module", autouse=True)
def _lib():
    try:
        L.load_host()
    except L.LibmHipError as e:
        pytest.fail(str(e))


@pytest.mark.parametrize("fn,v,dt", KINDS, ids=["-".join(k) for k in KINDS])
def test_host_consistent_within_bound(fn, v, dt):
    npdt = np.float64 if dt == "f64" else np.float32
    a = _inputs(fn, dt, 0)
    b = _inputs(fn, dt, 1)[::-1].copy() if fn in L.BINARY else None
    y = L.host_consistent(fn, a.astype(npdt), None if b is None else b.astype(npdt), v)
    rn, hi, lo = oracle.evaluate(fn, dt, a, b)
    if v == "exact":
        bad, idx = exact_compare(y.astype(np.float64), rn)
        assert bad == 0, "%s %s: x=%r y=%r want %r" % (fn, dt, a[idx[:3]], y[idx[:3]], rn[idx[:3]])
        return
    r = compare(y.astype(np.float64), rn, hi, lo, dt, BOUND[v])
    bad = r["bad_idx"][:4]
    assert r["violations"] == 0 and r["special_mismatch"] == 0, \
        "%s %s %s: x=%r y=%r want %r (max %.3f ulp)" % (fn, v, dt, a[bad], y[bad], rn[bad],
                                                       r["max_ulp"])


def test_cbrt_consistent_seed_over_the_reduced_range():
    """cbrt on a dense grid of the reduced argument range [0.5, 4) and its
    scalings, where the FMA-only seed and its Newton steps run."""
    m = np.linspace(0.5, 4.0, 3001)[:-1]
    x = np.concatenate([m, m * 2.0 ** 300, m * 2.0 ** -1050, -m * 2.0 ** -600])
    y = L.host_consistent("cbrt", x)
    rn, hi, lo = oracle.evaluate("cbrt", "f64", x)
    r = compare(y, rn, hi, lo, "f64", 1.0)
    assert r["violations"] == 0 and r["special_mismatch"] == 0, r["max_ulp"]


SUB_KINDS = [(fn, v, dt) for fn in W.SUBNORMAL_FNS for v in L.VARIANTS[fn] if v != "exact"
             for dt in ("f64", "f32")]


@pytest.mark.parametrize("fn,v,dt", SUB_KINDS, ids=["-".join(k) for k in SUB_KINDS])
def test_host_subnormal_results_bit_exact(fn, v, dt):
    """Arguments whose results lie in the subnormal range: every subnormal
    result equals the oracle's correctly rounded value bit for bit (the
    accurate paths of exp, exp2, exp10, pow, erf and erfc, and the
    tiny-argument identities of the others)."""
    npdt = np.float64 if dt == "f64" else np.float32
    a, b = W.subnormal_results(fn, dt, 3000, 0)
    y = L.host_consistent(fn, a.astype(npdt), None if b is None else b.astype(npdt), v)
    rn, hi, lo = oracle.evaluate(fn, dt, a.astype(np.float64),
                                 None if b is None else b.astype(np.float64))
    r = compare(y.astype(np.float64), rn, hi, lo, dt, BOUND[v], subnormal="exact")
    bad = r["bad_idx"][:4]
    assert r["subnormal_results"] >= 1000, r["subnormal_results"]
    assert r["violations"] == 0 and r["special_mismatch"] == 0, \
        "%s %s %s: %d subnormal mismatches; x=%r b=%r y=%r want %r" % (
            fn, v, dt, r["subnormal_mismatch"], a[bad], None if b is None else b[bad],
            y[bad], rn[bad])



@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_host_pow_over_the_whole_result_range(dt):
    """pow with |y log x| up to the overflow and underflow edges, where the
    logarithm's relative error is amplified ~745 times (binary64)."""
    npdt = np.float64 if dt == "f64" else np.float32
    a, b = W.pow_wide(dt, 6000, 0)
    y = L.host_consistent("pow", a.astype(npdt), b.astype(npdt), "u10")
    rn, hi, lo = oracle.evaluate("pow", dt, a.astype(np.float64), b.astype(np.float64))
    r = compare(y.astype(np.float64), rn, hi, lo, dt, 1.0)
    assert r["violations"] == 0 and r["special_mismatch"] == 0, (r["max_ulp"], a[r["bad_idx"][:3]],
                                                                 b[r["bad_idx"][:3]])


def test_erfc_subnormal_results_rounded_from_the_checked_pair():
    """erfc on [26.5, 27.3], where the binary64 result falls below 2^-1022:
    the main path rounds a subnormal result from its pair when the pair's
    error bound decides the rounding and leaves the rest to the accurate
    path.  Every subnormal result must be the correctly rounded one (a
    mis-decided rounding would be one unit off)."""
    x = np.random.default_rng(71).uniform(26.5, 27.3, 1500)
    y = L.host_consistent("erfc", x, None, "u10")
    rn, hi, lo = oracle.evaluate("erfc", "f64", x)
    sub = np.abs(rn) < 2.0 ** -1022
    assert sub.sum() > 1300
    bad = np.nonzero(y != rn)[0]
    assert bad.size == 0, (x[bad[:3]], y[bad[:3]], rn[bad[:3]])
