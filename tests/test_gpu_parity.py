"""GPU parity: every C-ABI entry point against the oracle, element by element.

Sizes span many 256-lane tiles plus a ragged tail; inputs are the seeded
workload mixtures (the mixture and its bf16/f16 form, large arguments, the
binary64 small set
at its full 2^20 size) plus the Annex F special set.  Bounds: 1.0 ULP (u10),
3.5 ULP (u35), bit-exact for fmod/remainder and for every NaN, +-inf and +-0
result, and for every subnormal result in binary64 and binary32 (the paper's
accuracy contract, Section 5, overview, read strictly for subnormals, and
its testers, Section 6); bf16, f16 and the binary32-through-binary64 form
report their subnormal mismatches and hold them to the bound.
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import check, run_gpu, run_oracle, to_device, BOUND
from tests.trig_hard_cases import mid_range, near_multiples

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402

N_PAR = 3 * 4096 + 37            # 24+ tiles of 512 f64 elements, ragged tail
CASES = [(fn, v, dt) for fn, v, dt, _ in L.all_entry_points()]
BINARY = L.BINARY


def _inputs(cfg, fn, dt, n, operand):
    base = "f32" if dt == "f32_via_f64" else dt
    if cfg == 2:
        return W.function_mixture(fn, base, n, operand)
    return W.large_args(fn, base, n, operand)


@pytest.fixture(scope="session", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    yield


@pytest.mark.parametrize("fn,variant,dt", CASES, ids=["-".join(c) for c in CASES])
def test_parity_mixture(fn, variant, dt):
    a = _inputs(2, fn, dt, N_PAR, 0)
    b = _inputs(2, fn, dt, N_PAR, 1) if fn in BINARY else None
    print("parity mixture", fn, variant, dt, flush=True)
    check(fn, variant, dt, a, b, label="mixture")


TRIG_CASES = [c for c in CASES if c[0] in ("sin", "cos", "tan", "fmod", "remainder")
              and c[2] in ("f64", "f32")]


@pytest.mark.parametrize("fn,variant,dt", TRIG_CASES, ids=["-".join(c) for c in TRIG_CASES])
def test_parity_large_arguments(fn, variant, dt):
    a = _inputs(3, fn, dt, N_PAR, 0)
    b = _inputs(3, fn, dt, N_PAR, 1) if fn in BINARY else None
    print("parity large arguments", fn, variant, dt, flush=True)
    check(fn, variant, dt, a, b, label="large_args")


HARD = [(fn, v, dt) for fn in ("sin", "cos", "tan") for v in ("u10", "u35")
        for dt in ("f64", "f32")]


@pytest.mark.parametrize("fn,variant,dt", HARD, ids=["-".join(c) for c in HARD])
def test_trig_reduction_hard_cases(fn, variant, dt):
    """Every float nearest to k pi/2 in the Cody-Waite range (binary64 below
    2^14, binary32 below 65536) and its neighbours: the smallest reduced
    arguments that range meets.  binary64 adds log-uniform arguments over
    [2^14, 1e14] (the Payne-Hanek range whose table rows have leading
    zeros)."""
    a = near_multiples(dt)
    if dt == "f64":
        a = np.concatenate([a, mid_range(8192)])
    print("trig hard cases", fn, variant, dt, a.size, flush=True)
    check(fn, variant, dt, a, label="hard cases")


@pytest.mark.parametrize("fn", ["sin", "cos", "exp", "log"])
def test_small_set_full(fn):
    """The binary64 small set at its full size: u10 on 2^20 elements."""
    a = W.small_set(fn)
    print("small set", fn, flush=True)
    res = check(fn, "u10", "f64", a, None, label="small_set")
    assert res["max_ulp"] <= 1.0


SPECIAL_F64 = [0.0, -0.0, math.inf, -math.inf, math.nan, 5e-324, -5e-324,
               2.2250738585072009e-308, -2.2250738585072009e-308, 2.2250738585072014e-308,
               1.0, -1.0, 0.5, -0.5, 2.0, -2.0, 3.0, -3.0, 1.7976931348623157e308,
               -1.7976931348623157e308, 709.782712893384, 709.7827128933841, -745.1332191019411,
               -745.1332191019412, 710.4758600739439, 1e-300, 1e22, 1e300, 0.75, 1.5,
               0.9999999999999999, -0.9999999999999999, 0.5000000000000001,
               -0.5000000000000001, 0.49999999999999994, 1.0000000000000002]


def _special_inputs(dt, binary):
    vals = np.array(SPECIAL_F64)
    if dt in ("f32", "f32_via_f64"):
        vals = np.concatenate([vals.astype(np.float32).astype(np.float64),
                               [1.401298464324817e-45, -1.401298464324817e-45,
                                1.1754942106924411e-38, 88.72283935546875, 88.72284, -103.97208,
                                89.41598, 3.4028234663852886e+38]])
    elif dt == "bf16":
        vals = W.round_to_bf16(vals.astype(np.float32)).astype(np.float64)
    elif dt == "f16":
        vals = np.concatenate([vals.astype(np.float16).astype(np.float64),
                               [2.0 ** -24, -(2.0 ** -24), 6.097555160522461e-05, 11.0859375,
                                65504.0]])
    # every value must be one of the format (the oracle sees exactly what the
    # kernel sees)
    if dt in ("f32", "f32_via_f64"):
        vals = vals.astype(np.float32).astype(np.float64)
    elif dt == "f16":
        vals = vals.astype(np.float16).astype(np.float64)
    elif dt == "bf16":
        vals = W.round_to_bf16(vals.astype(np.float32)).astype(np.float64)
    vals = np.unique(vals[~np.isnan(vals)])
    vals = np.concatenate([vals, [np.nan]])
    if binary:
        pairs = np.array(list(itertools.product(vals, vals)))
        return pairs[:, 0], pairs[:, 1]
    return vals, None


@pytest.mark.parametrize("fn,variant,dt", CASES, ids=["-".join(c) for c in CASES])
def test_special_values(fn, variant, dt):
    a, b = _special_inputs(dt, fn in BINARY)
    print("specials", fn, variant, dt, flush=True)
    check(fn, variant, dt, a, b, label="specials")


# ---------------------------------------------------------------------------
# boundary behaviour of the C-ABI
# ---------------------------------------------------------------------------
def test_abi_zero_length_and_null():
    assert L.libm_hip_sin_u10_f64(0, 0, 0, 0) == 0          # n == 0: OK, no launch
    assert L.libm_hip_sin_u10_f64(0, 0, 5, 0) == 1          # NULL with n > 0
    assert L.libm_hip_pow_u10_f32(0, 0, 0, 7, 0) == 1
    assert b"NULL" in L.load().libm_hip_last_error()


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16", "f16"])
def test_misaligned_in_place_and_streams(dt):
    """Unaligned views (scalar path), in-place calls, non-default stream."""
    n = 5000
    base = "f32" if dt == "f32_via_f64" else dt
    a = W.narrow_mixture("exp", base, n + 3, 9) if base in ("bf16", "f16") else \
        W.mixture("exp", base, n + 3, 9)
    ta = to_device(a, dt)
    view = ta[1:n + 1]                                       # 1-element offset
    assert view.data_ptr() % 16 != 0
    out = L.exp(view)
    want = L.exp(view.clone())
    torch.cuda.synchronize()
    assert torch.equal(out.view(torch.int8), want.view(torch.int8)) or \
        torch.equal(torch.nan_to_num(out.float(), nan=7.0), torch.nan_to_num(want.float(), nan=7.0))
    inplace = view.clone()
    L.exp(inplace, out=inplace)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        other = L.exp(view)
    s.synchronize()
    torch.cuda.synchronize()
    for t in (inplace, other):
        assert torch.equal(torch.nan_to_num(t.float(), nan=7.0),
                           torch.nan_to_num(want.float(), nan=7.0))


def test_generic_dispatcher_matches_named_entry():
    a = W.mixture("sin", "f64", 4096, 3)
    ta = to_device(a, "f64")
    out1 = L.sin(ta)
    out2 = torch.empty_like(ta)
    st = L.load().libm_hip_eval(0, 0, 0, ta.data_ptr(), None, out2.data_ptr(), ta.numel(), 0)
    assert st == 0
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(out1, nan=7.0), torch.nan_to_num(out2, nan=7.0))
    st = L.load().libm_hip_eval(0, 1, 2, ta.data_ptr(), None, out2.data_ptr(), 4, 0)
    assert st == 2                                           # u35 not served in bf16


# ---------------------------------------------------------------------------
# full benchmark size, sampled
# ---------------------------------------------------------------------------
FULL_NARROW = [("sin", "f16"), ("exp", "bf16"), ("tan", "bf16")]


@pytest.mark.parametrize("fn,dt", FULL_NARROW, ids=["-".join(c) for c in FULL_NARROW])
def test_full_size_sampled_narrow(fn, dt):
    """2^28 bf16/f16 elements (the narrow formats' benchmark size) through the
    narrow-format evaluators; 4096 sampled outputs checked against the
    oracle one by one."""
    n = 1 << 28
    a = W.narrow_mixture(fn, dt, n, 0)
    print("full size", fn, dt, flush=True)
    y = run_gpu(fn, "u10", dt, a)
    idx = np.concatenate([np.random.default_rng(6).integers(0, n, 4096), [0, n - 1]])
    from tests.ulp import compare
    rn, hi, lo = run_oracle(fn, dt, a[idx])
    res = compare(y[idx], rn, hi, lo, dt, 1.0)
    assert res["violations"] == 0 and res["special_mismatch"] == 0, res


POW_WIDE = [("u10", "f64"), ("u10", "f32"), ("u10", "f32_via_f64")]


@pytest.mark.parametrize("variant,dt", POW_WIDE, ids=["-".join(c) for c in POW_WIDE])
def test_pow_over_the_whole_result_range(variant, dt):
    """pow with |y log x| out to the overflow and underflow edges (where the
    logarithm's relative error is amplified the most), 2^16 + 37 pairs."""
    base = "f32" if dt == "f32_via_f64" else dt
    a, b = W.pow_wide(base, (1 << 16) + 37, 0)
    print("parity pow whole range", variant, dt, flush=True)
    check("pow", variant, dt, a, b, label="pow_wide")
