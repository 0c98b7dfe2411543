"""sincos: one pass, two outputs, each bit-identical to the sin and cos
entry points of the same variant and type (the Payne-Hanek elements are
reduced once and mapped twice).  The sin and cos entry points are checked
against the oracle elsewhere; here a sample is also checked against the
oracle directly.  Inputs: the mixture, the large-argument set, the special
values, a ragged tail and a misaligned view; the device-callable form too."""
import ctypes
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import to_device, to_host, run_oracle
from tests.ulp import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402

N = 3 * 4096 + 37
CASES = [(v, dt) for v, dt, _ in L.sincos_entry_points()]
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()


def _same(y0, y1):
    eq = (y0 == y1) & (np.signbit(y0) == np.signbit(y1))
    return eq | (np.isnan(y0) & np.isnan(y1))


def _inputs(dt, seed):
    base = "f32" if dt == "f32_via_f64" else dt
    a = W.function_mixture("sin", base, N, 70 + seed)
    if base in ("f64", "f32"):
        big = W.large_args("sin", base, N // 4, 71 + seed)
        a = np.concatenate([a, big])
    sp = W.specials(base)
    a[:sp.size] = sp
    return a


@pytest.mark.parametrize("v,dt", CASES, ids=["-".join(c) for c in CASES])
def test_sincos_matches_sin_and_cos(v, dt):
    a = _inputs(dt, 0)
    via = dt == "f32_via_f64"
    for shift in (0, 1):                      # 16-byte path, then the scalar one
        t = to_device(np.concatenate([a[:1], a]) if shift else a, dt)
        t = t[1:] if shift else t
        s, c = L.sincos(t, variant=v, via_f64=via)
        s_ref = L.evaluate("sin", t, variant=v, via_f64=via)
        c_ref = L.evaluate("cos", t, variant=v, via_f64=via)
        torch.cuda.synchronize()
        for got, want, what in ((s, s_ref, "sin"), (c, c_ref, "cos")):
            bad = ~_same(to_host(got), to_host(want))
            assert not bad.any(), "sincos %s %s (%s, shift %d): %d differ, e.g. x=%r" % (
                v, dt, what, shift, int(bad.sum()), a[np.nonzero(bad)[0][:3]])


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_sincos_against_oracle_sample(dt):
    a = _inputs(dt, 1)[:4000]
    t = to_device(a, dt)
    s, c = L.sincos(t)
    torch.cuda.synchronize()
    for fn, y in (("sin", s), ("cos", c)):
        rn, hi, lo = run_oracle(fn, dt, a)
        res = compare(to_host(y), rn, hi, lo, dt, 1.0)
        assert res["violations"] == 0 and res["special_mismatch"] == 0, (fn, dt, res["max_ulp"])


def test_sincos_in_place_and_zero_length():
    a = _inputs("f64", 2)
    t = to_device(a, "f64")
    c = torch.empty_like(t)
    s_ref = L.evaluate("sin", t)
    c_ref = L.evaluate("cos", t)
    L.sincos(t, outs=(t, c))                  # sin written over the input
    torch.cuda.synchronize()
    assert _same(to_host(t), to_host(s_ref)).all()
    assert _same(to_host(c), to_host(c_ref)).all()
    lib = L.load()
    assert lib.libm_hip_sincos_u10_f64(None, None, None, 0, None) == 0
    assert lib.libm_hip_sincos_u10_f64(t.data_ptr(), None, c.data_ptr(), 5, None) == 1


@pytest.mark.parametrize("v,dt", CASES, ids=["-".join(c) for c in CASES])
def test_sincos_device_api(v, dt):
    lib = ctypes.CDLL(os.path.join(HERE, "device_api", "libdevice_api_check.so"))
    vp = ctypes.c_void_p
    lib.device_api_sincos.restype = ctypes.c_int
    lib.device_api_sincos.argtypes = [ctypes.c_int, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp]
    a = _inputs(dt, 3)
    t = to_device(a, dt)
    via = dt == "f32_via_f64"
    s_ref, c_ref = L.sincos(t, variant=v, via_f64=via)
    s, c = torch.empty_like(t), torch.empty_like(t)
    st = lib.device_api_sincos(L.VARIANT_CODES[v], L.DTYPE_CODES[dt], t.data_ptr(), s.data_ptr(),
                               c.data_ptr(), t.numel(), torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    assert _same(to_host(s), to_host(s_ref)).all()
    assert _same(to_host(c), to_host(c_ref)).all()
