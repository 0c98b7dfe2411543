"""Results must not depend on which other elements share a wave or a
workgroup.

The paper selects one reduction per vector (Section 3.3); here every element
takes its own path, and the trig kernels gather their Payne-Hanek elements
across a workgroup.  Each case evaluates the same values in several
arrangements (as drawn, sorted so that whole waves take one path, reversed,
a single large argument among small ones, shifted by one element so the
vector and scalar paths swap) and requires bit-identical results after
undoing the arrangement.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import to_device, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402

N = 3 * 4096 + 37
TRIG = [(fn, v, dt) for fn in ("sin", "cos", "tan") for v in ("u10", "u35")
        for dt in ("f64", "f32")] + [(fn, "u10", dt) for fn in ("sin", "cos", "tan")
                                     for dt in ("bf16", "f16", "f32_via_f64")]
OTHERS = [(fn, "u10", dt) for fn in ("exp", "log", "pow", "atan2", "tanh", "asin", "acos")
          for dt in ("f64", "f32")] + [("atan", "u35", "f64"), ("acos", "u35", "f32"),
                                       ("log", "u35", "f64"), ("log10", "u10", "f32"),
                                       ("log1p", "u10", "f64"), ("exp10", "u10", "f32"),
                                       ("expm1", "u10", "f64"), ("cbrt", "u10", "f64"),
                                       ("hypot", "u10", "f64"), ("hypot", "u10", "f32"),
                                       ("atan2", "u35", "f64"), ("sinh", "u35", "f32"),
                                       ("tanh", "u35", "f64"), ("asinh", "u10", "f64"),
                                       ("acosh", "u10", "f32"), ("atanh", "u10", "f64"),
                                       ("erf", "u10", "f64"), ("erfc", "u10", "f32"),
                                       ("erfc", "u10", "f64"),
                                       ("fmod", "exact", "f64"), ("remainder", "exact", "f32"),
                                       ("fdim", "exact", "f64"), ("fmax", "exact", "f32")]
BINARY = L.BINARY
SLOW = {"f64": 2.0 ** 14, "f32": 65536.0, "bf16": 65536.0, "f16": 65536.0, "f32_via_f64": 2.0 ** 14}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()


def _inputs(fn, dt, operand):
    base = "f32" if dt == "f32_via_f64" else dt
    return W.function_mixture(fn, base, N, 40 + operand)


def _run(fn, v, dt, a, b):
    ta = to_device(a, dt)
    tb = to_device(b, dt) if b is not None else None
    out = L.evaluate(fn, ta, tb, variant=v, via_f64=(dt == "f32_via_f64"))
    torch.cuda.synchronize()
    return to_host(out)


def _same(y0, y1):
    eq = (y0 == y1) & (np.signbit(y0) == np.signbit(y1))
    eq |= np.isnan(y0) & np.isnan(y1)
    return eq


def _check_arrangements(fn, v, dt, a, b):
    y0 = _run(fn, v, dt, a, b)
    slow = ~(np.abs(a) < SLOW[dt])
    perms = {
        "sorted by path": np.argsort(slow, kind="stable"),
        "reversed": np.arange(N)[::-1].copy(),
        "random": np.random.default_rng(11).permutation(N),
    }
    for name, p in perms.items():
        y1 = _run(fn, v, dt, a[p], None if b is None else b[p])
        back = np.empty_like(y1)
        back[p] = y1
        bad = ~_same(y0, back)
        assert not bad.any(), "%s %s %s (%s): %d results differ, e.g. x=%r" % (
            fn, v, dt, name, int(bad.sum()), a[np.nonzero(bad)[0][:3]])
    # one element later: the 16-byte vector path becomes the scalar one
    a1 = np.concatenate([a[:1], a])
    b1 = None if b is None else np.concatenate([b[:1], b])
    ta = to_device(a1, dt)[1:]
    tb = None if b1 is None else to_device(b1, dt)[1:]
    y1 = to_host(L.evaluate(fn, ta, tb, variant=v, via_f64=(dt == "f32_via_f64")))
    torch.cuda.synchronize()
    bad = ~_same(y0, y1)
    assert not bad.any(), "%s %s %s (misaligned): %d results differ" % (fn, v, dt, int(bad.sum()))


@pytest.mark.parametrize("fn,v,dt", TRIG, ids=["-".join(c) for c in TRIG])
def test_trig_independent_of_neighbours(fn, v, dt):
    a = _inputs(fn, dt, 0)
    _check_arrangements(fn, v, dt, a, None)


@pytest.mark.parametrize("fn,v,dt", [c for c in TRIG if c[2] in ("f64", "f32")],
                         ids=["-".join(c) for c in TRIG if c[2] in ("f64", "f32")])
def test_single_large_argument_in_a_wave(fn, v, dt):
    """Waves of small arguments with exactly one Payne-Hanek element, waves
    with none and waves with all: every value matches its own result in a
    uniform array."""
    rng = np.random.default_rng(12)
    small = rng.uniform(-1e4, 1e4, N)
    big = np.where(rng.random(N) < 0.5, -1.0, 1.0) * 10.0 ** rng.uniform(15.0, 30.0, N)
    if dt == "f32":
        small, big = small.astype(np.float32), big.astype(np.float32)
    mixed = small.copy()
    mixed[17::128] = big[17::128]            # one large element per 128
    mixed[4096:4096 + 512] = big[4096:4096 + 512]
    y_mixed = _run(fn, v, dt, mixed, None)
    y_small = _run(fn, v, dt, small, None)
    y_big = _run(fn, v, dt, big, None)
    is_big = np.zeros(N, bool)
    is_big[17::128] = True
    is_big[4096:4096 + 512] = True
    want = np.where(is_big, y_big, y_small)
    bad = ~_same(y_mixed, want)
    assert not bad.any(), "%s %s %s: %d results depend on their neighbours" % (
        fn, v, dt, int(bad.sum()))


@pytest.mark.parametrize("fn,v,dt", OTHERS, ids=["-".join(c) for c in OTHERS])
def test_other_functions_independent_of_neighbours(fn, v, dt):
    a = _inputs(fn, dt, 0)
    b = _inputs(fn, dt, 1) if fn in BINARY else None
    _check_arrangements(fn, v, dt, a, b)
