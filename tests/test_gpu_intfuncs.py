"""ldexp, ilogb and frexp (C99 7.12.6) on the GPU against the oracle,
element by element and bit for bit, binary64 and binary32: the benchmark
mixture plus the special set, exponents uniform over the whole range and
near the overflow and subnormal edges, and a ragged length."""
import numpy as np
import pytest

import workloads as W
from oracle import intfuncs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402

N = 3 * 4096 + 37


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()


def _x(dt, seed):
    a = W.mixture("exp", dt, N, seed)
    sp = W.specials(dt)
    a[:sp.size] = sp
    return a


def _same(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    eq = (got == want) & (np.signbit(got) == np.signbit(want))
    return eq | (np.isnan(got) & np.isnan(want))


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_ldexp(dt):
    a = _x(dt, 31)
    lim = 2200 if dt == "f64" else 400
    rng = np.random.default_rng(32)
    e = rng.integers(-lim - 100, lim + 100, N).astype(np.int32)
    edge = 1024 if dt == "f64" else 128
    e[::3] = rng.integers(-edge - 60, edge + 5, e[::3].size)
    ta = torch.from_numpy(a).cuda()
    y = L.ldexp(ta, torch.from_numpy(e).cuda()).cpu().numpy()
    want = np.array([I.ldexp(float(v), int(k), dt) for v, k in zip(a, e)])
    bad = ~_same(y, want)
    assert not bad.any(), (a[bad][:3], e[bad][:3], y[bad][:3], want[bad][:3])


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_ilogb_frexp(dt):
    a = _x(dt, 33)
    ta = torch.from_numpy(a).cuda()
    e = L.ilogb(ta).cpu().numpy()
    m, fe = L.frexp(ta)
    m, fe = m.cpu().numpy(), fe.cpu().numpy()
    want_e = np.array([I.ilogb(float(v)) for v in a])
    assert (e == want_e).all(), a[e != want_e][:3]
    fr = [I.frexp(float(v)) for v in a]
    assert _same(m, [f[0] for f in fr]).all()
    assert (fe == np.array([f[1] for f in fr])).all()


def test_null_and_zero_length():
    lib = L.load()
    assert lib.libm_hip_ldexp_f64(None, None, None, 0, None) == 0
    assert lib.libm_hip_ldexp_f64(None, None, None, 3, None) == 1
    assert lib.libm_hip_ilogb_f32(None, None, 3, None) == 1
    assert lib.libm_hip_frexp_f64(None, None, None, 3, None) == 1


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_modf_lrint_lround(dt):
    a = _x(dt, 34)
    a[-64:] = np.array([0.5, -0.5, 1.5, -1.5, 2.5, -2.5, 1e19, -1e19, 9.2e18, -9.2e18] * 6 +
                       [0.49999997, -0.49999997, 4.5, 3.0], dtype=a.dtype)
    ta = torch.from_numpy(a).cuda()
    f, ip = L.modf(ta)
    want = [I.modf(float(v)) for v in a]
    assert _same(f.cpu().numpy(), [w[0] for w in want]).all()
    assert _same(ip.cpu().numpy(), [w[1] for w in want]).all()
    r = L.lrint(ta).cpu().numpy()
    assert (r == np.array([I.lrint(float(v)) for v in a], dtype=np.int64)).all()
    r = L.lround(ta).cpu().numpy()
    assert (r == np.array([I.lround(float(v)) for v in a], dtype=np.int64)).all()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_fma(dt):
    rng = np.random.default_rng(35)
    a, b, c = _x(dt, 36), _x(dt, 37)[::-1].copy(), _x(dt, 38)
    c[::4] = -(a[::4].astype(np.float64) * b[::4].astype(np.float64)).astype(a.dtype)  # cancellation
    sp = W.specials(dt)
    trip = np.array([(x, y, z) for x in sp for y in sp for z in sp], dtype=a.dtype)
    a = np.concatenate([a, trip[:, 0]])
    b = np.concatenate([b, trip[:, 1]])
    c = np.concatenate([c, trip[:, 2]])
    ta, tb, tc = (torch.from_numpy(np.ascontiguousarray(v)).cuda() for v in (a, b, c))
    y = L.fma(ta, tb, tc).cpu().numpy()
    want = np.array([I.fma(float(x), float(yv), float(z), dt) for x, yv, z in zip(a, b, c)])
    bad = ~_same(y, want)
    assert not bad.any(), (a[bad][:3], b[bad][:3], c[bad][:3], y[bad][:3], want[bad][:3])


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_remquo(dt):
    """remquo against the oracle: the remainder bit for bit (and equal to
    the remainder entry point), the quotient's sign and low three bits."""
    a = np.concatenate([W.large_args("fmod", dt, N, 40), _x(dt, 41)])
    b = np.concatenate([W.large_args("fmod", dt, N, 42), _x(dt, 43)[::-1]])
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    r, q = L.remquo(ta, tb)
    r, q = r.cpu().numpy(), q.cpu().numpy()
    want = [I.remquo(float(u), float(v)) for u, v in zip(a, b)]
    assert _same(r, [w[0] for w in want]).all()
    assert _same(r, L.remainder(ta, tb).cpu().numpy()).all()
    wq = np.array([w[1] for w in want], dtype=np.int32)
    bad = q != wq
    assert not bad.any(), (a[bad][:3], b[bad][:3], q[bad][:3], wq[bad][:3])
