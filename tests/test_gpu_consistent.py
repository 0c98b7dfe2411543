"""Bit-identity of the GPU and host builds of the bit-consistent form (the
paper's bit-consistent functions and its third tester, which compares an
MD5 digest of all outputs across platforms; Section 3.3, Section 6).

Every (function, variant) in binary64 and binary32: libm_hip_consistent_eval
on the GPU and libm_hip_host_eval on the host get the same inputs (the
function's benchmark mixture, the special set, huge trigonometric arguments
and, for the trig functions, doubles nearest to multiples of pi/2); every
output must be bit-identical, NaNs aside, which compare equal whatever their
payload (C99 leaves the payload of a generated NaN open).  One MD5 over all
outputs of both sides closes the test.  The GPU outputs themselves are
checked against the oracle on ORACLE_N elements from each end of the input
(the special set and the mixture at the front; for the trig functions the
doubles nearest to multiples of pi/2 and the mid-range points at the back)."""
import hashlib

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import check_values, to_device
from tests.trig_hard_cases import mid_range, near_multiples

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402

N = 1 << 16
ORACLE_N = 3072
KINDS = [(fn, v, dt) for fn in L.UNARY + L.BINARY for v in L.VARIANTS[fn]
         for dt in ("f64", "f32")]
DIGEST = {"gpu": hashlib.md5(), "host": hashlib.md5()}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    L.load_host()


def _inputs(fn, dt, operand):
    a = W.function_mixture(fn, dt, N, 700 + operand)
    sp = W.specials(dt)
    a[:sp.size] = sp
    if fn in ("sin", "cos", "tan") and operand == 0:
        big = W.large_args(fn, dt, N // 4, 710)
        a[sp.size:sp.size + big.size] = big
        h = near_multiples(dt)
        h = np.concatenate([h[::max(1, h.size // 8192)][:8192], mid_range(4096)])
        a[-h.size:] = h
    return a


def _canon(y):
    """bytes of y with every NaN replaced by one quiet NaN"""
    y = y.copy()
    y[np.isnan(y)] = np.nan
    return y.tobytes()


@pytest.mark.parametrize("fn,v,dt", KINDS, ids=["-".join(k) for k in KINDS])
def test_gpu_matches_host_bit_for_bit(fn, v, dt):
    npdt = np.float64 if dt == "f64" else np.float32
    a = _inputs(fn, dt, 0).astype(npdt)
    b = _inputs(fn, dt, 1).astype(npdt) if fn in L.BINARY else None
    ta = to_device(a, dt)
    tb = to_device(b, dt) if b is not None else None
    g = L.consistent(fn, ta, tb, v)
    torch.cuda.synchronize()
    yg = g.cpu().numpy()
    yh = L.host_consistent(fn, a, b, v)
    same = (yg.view(np.uint64 if dt == "f64" else np.uint32) ==
            yh.view(np.uint64 if dt == "f64" else np.uint32)) | (np.isnan(yg) & np.isnan(yh))
    bad = np.nonzero(~same)[0]
    assert bad.size == 0, "%s %s %s: %d of %d differ, e.g. x=%r gpu=%r host=%r" % (
        fn, v, dt, bad.size, a.size, a[bad[:3]], yg[bad[:3]], yh[bad[:3]])
    k = ORACLE_N
    sel = np.r_[0:k, N - k:N]
    check_values(fn, v, dt, a[sel].astype(np.float64),
                 None if b is None else b[sel].astype(np.float64),
                 yg[sel].astype(np.float64), label="consistent")
    DIGEST["gpu"].update(_canon(yg))
    DIGEST["host"].update(_canon(yh))
    # the default entry point: the same bounds, but hardware estimates may
    # move the last bit of some results
    d = L.evaluate(fn, ta, tb, variant=v).cpu().numpy()
    agree = np.mean((d == yg) | (np.isnan(d) & np.isnan(yg)))
    print("consistent %s %s %s: bit-identical to the host; %.5f identical to the default "
          "entry point" % (fn, v, dt, agree), flush=True)


def test_md5_of_all_outputs_agrees():
    gd, hd = DIGEST["gpu"].hexdigest(), DIGEST["host"].hexdigest()
    print("md5 gpu %s host %s" % (gd, hd), flush=True)
    assert gd == hd


def test_consistent_rejects_narrow_types_and_unknown_functions():
    lib = L.load()
    st = lib.libm_hip_consistent_eval(L.FN_CODES["exp"], 0, L.DTYPE_CODES["bf16"], None, None,
                                      None, 4, None)
    assert st == 2
    assert lib.libm_hip_consistent_eval(L.FN_CODES["exp"], 1, 0, None, None, None, 4, None) == 2
    assert lib.libm_hip_consistent_eval(L.FN_CODES["exp"], 0, 0, None, None, None, 0, None) == 0
    assert lib.libm_hip_consistent_eval(L.FN_CODES["exp"], 0, 0, None, None, None, 4, None) == 1
