"""libm_hip_batch_run_noalloc (the batched evaluation with its request table
in the library's fixed device array) against libm_hip_batch_run with a plan:
bit-identical outputs on two calls in a row, the second with fewer and
shorter requests (the array keeps the first call's contents, so the second
must not read any of them), then the limit of 256 requests."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import to_device

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()


def _requests(k, hi, seed):
    reqs = []
    for fn, var, dt, n, idx in W.batch_requests(k, 3.0, hi)[:k]:
        a, b = W.request_inputs(fn, dt, n, idx + seed)
        ta = to_device(a, dt)
        tb = to_device(b, dt) if b is not None else None
        reqs.append((fn, var, dt, ta, tb, torch.empty_like(ta)))
    return reqs


def _same(x, y):
    x = x.float() if x.dtype in (torch.bfloat16, torch.float16) else x
    y = y.float() if y.dtype in (torch.bfloat16, torch.float16) else y
    return torch.equal(torch.nan_to_num(x, nan=7.0), torch.nan_to_num(y, nan=7.0)) and \
        torch.equal(torch.isnan(x), torch.isnan(y))


@pytest.mark.parametrize("k,hi,seed", [(64, 5.5, 0), (9, 4.0, 500)])
def test_noalloc_matches_plan(k, hi, seed):
    print("noalloc batch", k, hi, flush=True)
    reqs = _requests(k, hi, seed)
    plan = L.BatchPlan(64, use_graph=True)
    plan.run(reqs)
    torch.cuda.synchronize()
    want = [out.clone() for *_, out in reqs]
    for *_, out in reqs:
        out.fill_(0)
    L.batch_run_noalloc(reqs)
    torch.cuda.synchronize()
    for (fn, v, dt, a, b, out), w in zip(reqs, want):
        assert _same(out, w), (fn, v, dt, a.numel())
    plan.close()


def test_noalloc_two_calls_second_smaller():
    first = _requests(40, 5.5, 1000)
    second = _requests(5, 3.6, 2000)
    for reqs in (first, second):
        ref = [L.evaluate(fn, a, b, variant=v, via_f64=(dt == "f32_via_f64"))
               for fn, v, dt, a, b, out in reqs]
        L.batch_run_noalloc(reqs)
        torch.cuda.synchronize()
        for (fn, v, dt, a, b, out), r in zip(reqs, ref):
            assert _same(out, r), (fn, v, dt, a.numel())


def test_noalloc_limits_and_errors():
    lib = L.load()
    a = to_device(W.mixture("exp", "f64", 1000, 0), "f64")
    out = torch.empty_like(a)
    reqs = [("exp", "u10", "f64", a, None, out)] * 257
    arr = L.request_array(reqs)
    assert lib.libm_hip_batch_run_noalloc(arr, 257, None) == 1
    assert b"256" in lib.libm_hip_last_error()
    assert lib.libm_hip_batch_run_noalloc(arr, 0, None) == 0
    bad = L.request_array([("fmod", "u10", "f64", a, a, out)])
    bad[0].variant = L.VARIANT_CODES["u10"]
    assert lib.libm_hip_batch_run_noalloc(bad, 1, None) == 2
    # 256 requests is the limit and is served
    reqs = [("exp", "u10", "f64", a, None, out)] * 256
    L.batch_run_noalloc(reqs)
    torch.cuda.synchronize()
    assert _same(out, L.evaluate("exp", a))
