"""Sweeps over whole input formats (the paper's testers check random bit
patterns and regular grids, Section 6; a GPU can afford every pattern).

* binary32: every STRIDE-th bit pattern (default stride 61, an odd step so
  every residue of the low mantissa bits is visited; LIBM_HIP_SWEEP_STRIDE=1
  sweeps all 2^32) for sin u10/u35, cos, tan, exp, log u10/u35, asin u10/u35, acos,
  atan u10/u35, log10, log1p, exp10, expm1, cbrt, asinh, acosh, atanh, erf,
  erfc, and sinh, cosh, tanh u35.
  The host's
  binary64 functions screen the results (their error, at most a few binary64
  ulps, is below 1e-7 binary32 ulp); every element the screen cannot clear
  (estimated error within 1e-4 of the bound, a special-class difference, or a
  subnormal/zero/infinite result different from the rounded binary64 value)
  is decided by the oracle.
* bf16 and f16: all 65 536 patterns of every unary u10 function against the
  oracle directly.
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest
import scipy.special as sps

from tests.gpu_common import run_gpu, run_oracle, to_device, to_host, BOUND
from tests.ulp import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402

STRIDE = int(os.environ.get("LIBM_HIP_SWEEP_STRIDE", "61"))
CHUNK = 1 << 24
NP_F = {"sin": np.sin, "cos": np.cos, "tan": np.tan, "exp": np.exp, "log": np.log,
        "asin": np.arcsin, "acos": np.arccos, "atan": np.arctan, "log10": np.log10,
        "log1p": np.log1p, "exp10": lambda x: np.power(10.0, x), "expm1": np.expm1,
        "cbrt": np.cbrt, "sinh": np.sinh, "cosh": np.cosh, "tanh": np.tanh,
        "asinh": np.arcsinh, "acosh": np.arccosh, "atanh": np.arctanh, "erf": sps.erf,
        "erfc": sps.erfc}
SWEEP = [("sin", "u10"), ("sin", "u35"), ("cos", "u10"), ("tan", "u10"), ("exp", "u10"),
         ("log", "u10"), ("log", "u35"), ("asin", "u10"), ("asin", "u35"), ("acos", "u10"),
         ("atan", "u10"), ("atan", "u35"), ("log10", "u10"), ("log1p", "u10"),
         ("exp10", "u10"), ("expm1", "u10"), ("cbrt", "u10"), ("sinh", "u35"),
         ("cosh", "u35"), ("tanh", "u35"), ("asinh", "u10"), ("acosh", "u10"),
         ("atanh", "u10"), ("erf", "u10"), ("erfc", "u10")]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()


def _host_ref(f, x64):
    """binary64 reference over a thread pool (numpy releases the GIL)."""
    parts = np.array_split(x64, 16)
    with np.errstate(all="ignore"), cf.ThreadPoolExecutor(16) as ex:
        return np.concatenate(list(ex.map(f, parts)))


def _screen(y, ref, bound):
    """Indices the binary64 screen cannot clear."""
    with np.errstate(all="ignore"):
        rn = ref.astype(np.float32).astype(np.float64)
        tiny = 2.0 ** -126
        e = np.maximum(np.frexp(np.abs(ref))[1].astype(np.int64) - 1, -126)
        ulp = np.ldexp(1.0, (e - 23).astype(np.int32))
        err = np.abs(y - ref) / ulp
        finite = np.isfinite(y) & np.isfinite(rn)
        same = (y == rn) & (np.signbit(y) == np.signbit(rn))
        same |= np.isnan(y) & np.isnan(rn)
        flag = finite & ~(err <= bound - 1e-4)
        flag |= ~finite & ~same
        flag |= ((np.abs(rn) < tiny) | (np.abs(y) < tiny)) & ~same
        ok = finite & ~flag
        est = float(err[ok].max()) if ok.any() else 0.0
    return np.nonzero(flag)[0], est


@pytest.mark.parametrize("fn,variant", SWEEP, ids=["-".join(c) for c in SWEEP])
def test_binary32_sweep(fn, variant):
    bound = BOUND[variant]
    total = flagged = 0
    worst = est_max = 0.0
    for ci, start in enumerate(range(0, 1 << 32, CHUNK * STRIDE)):
        if ci and ci % 32 == 0:
            print("  sweep %s %s: %d patterns so far" % (fn, variant, total), flush=True)
        stop = min(start + CHUNK * STRIDE, 1 << 32)
        bits = np.arange(start, stop, STRIDE, dtype=np.uint64).astype(np.uint32)
        x32 = bits.view(np.float32)
        xd = torch.from_numpy(x32).cuda()
        yd = L.evaluate(fn, xd, variant=variant)
        torch.cuda.synchronize()
        y = yd.cpu().numpy().astype(np.float64)
        x64 = x32.astype(np.float64)
        ref = _host_ref(NP_F[fn], x64)
        idx, est = _screen(y, ref, bound)
        est_max = max(est_max, est)
        total += bits.size
        if idx.size:
            flagged += idx.size
            assert idx.size < 100000, "%s %s: %d elements not cleared by the screen" % (
                fn, variant, idx.size)
            rn, hi, lo = run_oracle(fn, "f32", x64[idx])
            res = compare(y[idx], rn, hi, lo, "f32", bound)
            bad = res["bad_idx"][:4]
            assert res["violations"] == 0 and res["special_mismatch"] == 0, \
                "%s %s: x=%r y=%r want %r (max %.3f ulp)" % (
                    fn, variant, x64[idx][bad], y[idx][bad], rn[bad], res["max_ulp"])
            worst = max(worst, res["max_ulp"])
    print("sweep %s %s f32: %d patterns (stride %d), max error %.4f ulp (binary64 screen), "
          "%d decided by the oracle, worst of those %.3f ulp"
          % (fn, variant, total, STRIDE, est_max, flagged, worst), flush=True)


NARROW_UNARY = ["sin", "cos", "tan", "exp", "exp2", "log", "log2", "sinh", "cosh", "tanh",
                "asin", "acos", "atan", "log10", "log1p", "exp10", "expm1", "cbrt", "asinh",
                "acosh", "atanh", "erf", "erfc"]


@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("fn", NARROW_UNARY)
def test_narrow_all_patterns(fn, dt):
    bits = np.arange(1 << 16, dtype=np.uint32)
    if dt == "bf16":
        x = (bits << 16).view(np.float32).astype(np.float64)
    else:
        x = bits.astype(np.uint16).view(np.float16).astype(np.float64)
    y = run_gpu(fn, "u10", dt, x)
    rn, hi, lo = run_oracle(fn, dt, x)
    res = compare(y, rn, hi, lo, dt, 1.0)
    bad = res["bad_idx"][:4]
    assert res["violations"] == 0 and res["special_mismatch"] == 0, \
        "%s %s: x=%r y=%r want %r (max %.3f ulp)" % (fn, dt, x[bad], y[bad], rn[bad],
                                                    res["max_ulp"])
    print("all %s patterns %s: max %.3f ulp" % (dt, fn, res["max_ulp"]), flush=True)


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_narrow_pow_pairs(dt):
    """pow on 2^18 pairs of the format: half random bit patterns for both
    operands, half bases within 20 % of 1 with exponents U[-40, 40] rounded
    to 0.1 (the region where y log2 x stays finite and is most sensitive to
    the logarithm's accuracy), against the oracle."""
    n = 1 << 18
    rng = np.random.default_rng(17)
    bits = rng.integers(0, 1 << 16, size=(2, n)).astype(np.uint32)
    if dt == "bf16":
        pat = (bits << 16).view(np.float32).astype(np.float64)
    else:
        pat = bits.astype(np.uint16).view(np.float16).astype(np.float64)
    near = rng.random(n) < 0.5
    x = np.where(near, 1.0 + rng.uniform(-0.2, 0.2, n), pat[0])
    y = np.where(near, np.round(rng.uniform(-40.0, 40.0, n), 1), pat[1])
    base = {"bf16": "bf16", "f16": "f16"}[dt]
    x = to_host(to_device(x, base))          # exact values of the format
    y = to_host(to_device(y, base))
    r = run_gpu("pow", "u10", dt, x, y)
    rn, hi, lo = run_oracle("pow", dt, x, y)
    res = compare(r, rn, hi, lo, dt, 1.0)
    bad = res["bad_idx"][:4]
    assert res["violations"] == 0 and res["special_mismatch"] == 0, \
        "pow %s: x=%r y=%r got %r want %r (max %.3f ulp)" % (dt, x[bad], y[bad], r[bad], rn[bad],
                                                           res["max_ulp"])
    print("pow %s pairs: max %.3f ulp" % (dt, res["max_ulp"]), flush=True)


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_narrow_atan2_pairs(dt):
    """atan2 on 2^18 pairs of the format: random bit patterns for both
    operands (every sign, zero, infinity, NaN and subnormal combination
    occurs), a quarter of them with y/x near 1 where the octant changes,
    against the oracle."""
    n = 1 << 18
    rng = np.random.default_rng(29)
    bits = rng.integers(0, 1 << 16, size=(2, n)).astype(np.uint32)
    if dt == "bf16":
        pat = (bits << 16).view(np.float32).astype(np.float64)
    else:
        pat = bits.astype(np.uint16).view(np.float16).astype(np.float64)
    near = rng.random(n) < 0.25
    y = pat[0]
    x = np.where(near, y * rng.uniform(0.9, 1.1, n) * rng.choice([-1.0, 1.0], n), pat[1])
    x = to_host(to_device(x, dt))
    y = to_host(to_device(y, dt))
    r = run_gpu("atan2", "u10", dt, y, x)
    rn, hi, lo = run_oracle("atan2", dt, y, x)
    res = compare(r, rn, hi, lo, dt, 1.0)
    bad = res["bad_idx"][:4]
    assert res["violations"] == 0 and res["special_mismatch"] == 0, \
        "atan2 %s: y=%r x=%r got %r want %r (max %.3f ulp)" % (dt, y[bad], x[bad], r[bad], rn[bad],
                                                             res["max_ulp"])
    print("atan2 %s pairs: max %.3f ulp" % (dt, res["max_ulp"]), flush=True)


def test_sqrt_correctly_rounded_sweep():
    """sqrt (exact variant: the correctly rounded square root) on every
    STRIDE-th binary32 pattern against numpy's binary32 square root (an IEEE
    operation), and on 2^22 random binary64 patterns against the host's;
    bit for bit, NaN as a class."""
    total = bad = 0
    for start in range(0, 1 << 32, CHUNK * STRIDE):
        bits = np.arange(start, min(start + CHUNK * STRIDE, 1 << 32), STRIDE, dtype=np.uint64)
        x = bits.astype(np.uint32).view(np.float32)
        y = run_gpu("sqrt", "exact", "f32", x.astype(np.float64)).astype(np.float32)
        with np.errstate(invalid="ignore"):
            want = np.sqrt(x)
        same = (y.view(np.uint32) == want.view(np.uint32)) | (np.isnan(y) & np.isnan(want))
        bad += int((~same).sum())
        total += x.size
    assert bad == 0, "%d of %d binary32 square roots differ" % (bad, total)
    rng = np.random.default_rng(23)
    x = rng.integers(0, 1 << 63, 1 << 22, dtype=np.uint64).view(np.float64)
    y = run_gpu("sqrt", "exact", "f64", x)
    with np.errstate(invalid="ignore"):
        want = np.sqrt(x)
    same = (y.view(np.uint64) == want.view(np.uint64)) | (np.isnan(y) & np.isnan(want))
    assert same.all(), x[~same][:4]
    print("sqrt: %d binary32 patterns and 2^22 binary64 ones correctly rounded" % total,
          flush=True)
