"""Batched persistent kernel (one hip-graph replay per run) against the
per-function entry points: bit-identical outputs on the 64-request mix
(function, variant and dtype drawn uniformly, lengths log-uniform), graph
replays interleaved with eager work, the direct-launch mode, and the
validation errors."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402


@pytest.fixture(scope="session", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()


def _requests(hi=5.3):
    reqs = []
    for fn, var, dt, n, idx in W.batch_requests(64, 3.0, hi):
        a, b = W.request_inputs(fn, dt, n, idx)
        ta = to_device(a, dt)
        tb = to_device(b, dt) if b is not None else None
        reqs.append((fn, var, dt, ta, tb, torch.empty_like(ta)))
    return reqs


def _same(x, y):
    x = x.float() if x.dtype in (torch.bfloat16, torch.float16) else x
    y = y.float() if y.dtype in (torch.bfloat16, torch.float16) else y
    return torch.equal(torch.nan_to_num(x, nan=7.0), torch.nan_to_num(y, nan=7.0)) and \
        torch.equal(torch.isnan(x), torch.isnan(y))


def _reference(reqs):
    return [L.evaluate(fn, a, b, variant=v, via_f64=(dt == "f32_via_f64"))
            for fn, v, dt, a, b, out in reqs]


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_bit_identical_to_per_function(use_graph):
    reqs = _requests()
    ref = _reference(reqs)
    plan = L.BatchPlan(64, use_graph=use_graph)
    plan.run(reqs)
    torch.cuda.synchronize()
    for (fn, v, dt, a, b, out), r in zip(reqs, ref):
        assert _same(out, r), (fn, v, dt, a.numel())
    plan.close()


def test_graph_replays_with_eager_work_between():
    reqs = _requests(4.5)
    ref = _reference(reqs)
    plan = L.BatchPlan(64, use_graph=True)
    for rep in range(4):
        for *_, out in reqs:
            out.fill_(123.0)
        junk = torch.randn(1 << 20, device="cuda").sum()     # eager work
        plan.run(reqs)
        torch.cuda.synchronize()
        assert junk.isfinite()
        for (fn, v, dt, a, b, out), r in zip(reqs, ref):
            assert _same(out, r), (rep, fn, v, dt)
    # a different request list through the same captured graph
    reqs2 = list(reversed(reqs[:20]))
    for *_, out in reqs2:
        out.zero_()
    plan.run(reqs2)
    torch.cuda.synchronize()
    for (fn, v, dt, a, b, out) in reqs2:
        assert _same(out, L.evaluate(fn, a, b, variant=v, via_f64=(dt == "f32_via_f64")))
    plan.close()


def test_batch_validation_errors():
    plan = L.BatchPlan(4)
    x = torch.ones(8, dtype=torch.bfloat16, device="cuda")
    with pytest.raises(L.LibmHipError):                 # u35 is not served in bf16
        plan.run([("sin", "u35", "bf16", x, None, x)])
    y = torch.ones(8, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LibmHipError):                 # more requests than the plan holds
        plan.run([("exp", "u10", "f64", y, None, y)] * 5)
    plan.run([])                                        # empty list: nothing to do
    plan.close()


def test_batch_inverse_trig_and_log_u35_requests():
    """asin, acos, atan in every served variant and dtype, and log u35,
    through one plan."""
    reqs = []
    kinds = [(f, v, d) for f in ("asin", "acos", "atan") for v in ("u10", "u35")
             for d in ("f64", "f32", "bf16", "f16", "f32_via_f64")
             if v == "u10" or d in ("f64", "f32")]
    kinds += [("log", "u35", "f64"), ("log", "u35", "f32")]
    for i, (fn, v, dt) in enumerate(kinds):
        base = "f32" if dt == "f32_via_f64" else dt
        a = W.function_mixture(fn, base, 5000 + 997 * i, 300 + i)
        ta = to_device(a, dt)
        reqs.append((fn, v, dt, ta, None, torch.empty_like(ta)))
    ref = _reference(reqs)
    plan = L.BatchPlan(64, use_graph=True)
    plan.run(reqs)
    torch.cuda.synchronize()
    for (fn, v, dt, a, b, out), r in zip(reqs, ref):
        assert _same(out, r), (fn, v, dt)
    plan.close()


def test_batch_c99_function_requests():
    """log10, log1p, exp10, expm1, cbrt, hypot, asinh, acosh, atanh, erf and
    erfc in every dtype through one plan (hypot binary), against the per-function
    entry points."""
    reqs = []
    kinds = [(f, d) for f in ("log10", "log1p", "exp10", "expm1", "cbrt", "hypot", "asinh",
                              "acosh", "atanh", "erf", "erfc")
             for d in ("f64", "f32", "bf16", "f16", "f32_via_f64")]
    for i, (fn, dt) in enumerate(kinds):
        base = "f32" if dt == "f32_via_f64" else dt
        a = W.function_mixture(fn, base, 4000 + 991 * i, 400 + i)
        ta = to_device(a, dt)
        tb = None
        if fn == "hypot":
            tb = to_device(W.function_mixture(fn, base, a.size, 450 + i), dt)
        reqs.append((fn, "u10", dt, ta, tb, torch.empty_like(ta)))
    ref = _reference(reqs)
    plan = L.BatchPlan(64, use_graph=True)
    plan.run(reqs)
    torch.cuda.synchronize()
    for (fn, v, dt, a, b, out), r in zip(reqs, ref):
        assert _same(out, r), (fn, v, dt)
    plan.close()


def test_batch_exact_function_requests():
    """fmod, remainder, fdim, fmax and fmin (exact, binary64 and binary32)
    through one plan, against the per-function entry points."""
    reqs = []
    kinds = [(f, d) for f in ("fmod", "remainder", "fdim", "fmax", "fmin") for d in ("f64", "f32")]
    for i, (fn, dt) in enumerate(kinds):
        a = W.function_mixture(fn, dt, 3000 + 977 * i, 500 + i)
        b = W.function_mixture(fn, dt, a.size, 550 + i)
        ta, tb = to_device(a, dt), to_device(b, dt)
        reqs.append((fn, "exact", dt, ta, tb, torch.empty_like(ta)))
    ref = _reference(reqs)
    plan = L.BatchPlan(64, use_graph=True)
    plan.run(reqs)
    torch.cuda.synchronize()
    for (fn, v, dt, a, b, out), r in zip(reqs, ref):
        assert _same(out, r), (fn, v, dt)
    plan.close()


def test_plan_on_an_explicit_device_and_error_channel():
    """A plan made for device 0 by number runs like one on the current
    device; an unsupported request is reported on libm_hip_last_error."""
    import ctypes
    a = to_device(W.mixture("exp", "f64", 10000, 0), "f64")
    out = torch.empty_like(a)
    plan = L.BatchPlan(4, use_graph=False, device=0)
    plan.run([("exp", "u10", "f64", a, None, out)])
    torch.cuda.synchronize()
    assert _same(out, L.evaluate("exp", a))
    lib = L.load()
    arr = (L.Request * 1)(L.Request(L.FN_CODES["fmod"], L.VARIANT_CODES["u10"], 0, 0,
                                    a.data_ptr(), a.data_ptr(), out.data_ptr(), 16))
    assert plan.run_raw(arr, 1, 0) == 2
    assert b"unsupported" in lib.libm_hip_last_error()
    bad = ctypes.c_void_p()
    n = torch.cuda.device_count()
    assert lib.libm_hip_batch_plan_create(ctypes.byref(bad), 4, n) == 1
    plan.close()
