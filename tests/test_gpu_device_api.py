"""The device-callable API (include/libm_hip_device.h) gives the same bits as
the entry points, and its results meet the oracle's bounds (checked
directly on the first ORACLE_N outputs of every case, special values
included).

The check library (tests/device_api/check.hip, built by build()) runs the
header's functions in a plain one-element-per-lane kernel compiled with the
compiler's default floating-point contraction, so this also checks that the
evaluator headers keep their own contraction control.  Inputs: the mixtures
(every served function, variant and dtype) and the special-value set.
"""
import ctypes
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import check_values, to_device, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "device_api", "libdevice_api_check.so")
CASES = [(fn, v, dt) for fn, v, dt, _ in L.all_entry_points()]
BINARY = L.BINARY
N = 3 * 4096 + 37
ORACLE_N = 4096


@pytest.fixture(scope="module")
def chk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(LIB):
        raise RuntimeError("%s is missing: run __graft_entry__.build()" % LIB)
    L.load()
    lib = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    lib.device_api_eval.restype = ctypes.c_int
    lib.device_api_eval.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                    ctypes.c_size_t, vp]
    lib.device_api_masked_sin.restype = ctypes.c_int
    lib.device_api_masked_sin.argtypes = [vp, vp, ctypes.c_size_t, vp]
    return lib


def _same(y0, y1):
    eq = (y0 == y1) & (np.signbit(y0) == np.signbit(y1))
    return eq | (np.isnan(y0) & np.isnan(y1))


def _inputs(fn, dt, operand):
    base = "f32" if dt == "f32_via_f64" else dt
    a = W.function_mixture(fn, base, N, 60 + operand)
    sp = W.specials(base)
    a[:sp.size] = sp
    return a


@pytest.mark.parametrize("fn,v,dt", CASES, ids=["-".join(c) for c in CASES])
def test_device_api_matches_entry_point(chk, fn, v, dt):
    a = _inputs(fn, dt, 0)
    b = _inputs(fn, dt, 1) if fn in BINARY else None
    ta = to_device(a, dt)
    tb = to_device(b, dt) if b is not None else None
    want = L.evaluate(fn, ta, tb, variant=v, via_f64=(dt == "f32_via_f64"))
    got = torch.empty_like(ta)
    st = chk.device_api_eval(L.FN_CODES[fn], L.VARIANT_CODES[v], L.DTYPE_CODES[dt],
                             ta.data_ptr(), None if tb is None else tb.data_ptr(),
                             got.data_ptr(), N, torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    y0, y1 = to_host(want), to_host(got)
    bad = ~_same(y0, y1)
    assert not bad.any(), "%s %s %s: %d differ, e.g. x=%r" % (fn, v, dt, int(bad.sum()),
                                                            a[np.nonzero(bad)[0][:3]])
    k = ORACLE_N
    check_values(fn, v, dt, a[:k], None if b is None else b[:k], y1[:k], label="device_api")


def test_masked_evaluation(chk):
    a = _inputs("sin", "f64", 0)
    ta = to_device(a, "f64")
    got = torch.empty_like(ta)
    st = chk.device_api_masked_sin(ta.data_ptr(), got.data_ptr(), N,
                                   torch.cuda.current_stream().cuda_stream)
    assert st == 0
    want = to_host(L.evaluate("sin", ta, variant="u10"))
    y = to_host(got)
    even = np.arange(N) % 2 == 0
    assert _same(y[even], want[even]).all()
    assert _same(y[~even], a[~even]).all()
