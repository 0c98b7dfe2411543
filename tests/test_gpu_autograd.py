"""Backward kernels and torch.autograd.Function wrappers on the GPU.

* g * f'(x) against the oracle's correctly rounded derivative products:
  within 2.5 ULP for sin, cos, tan, exp, log, tanh and 4 ULP for the pow and
  atan2 partials (binary32 and binary64);
* autograd through the wrappers against central finite differences of the
  forward kernels (binary64) and torch.autograd.gradcheck;
* the autograd workload at its full size (2^24 binary32 elements,
  x ~ U[0.1, 10]) with 4096 sampled gradients checked against the oracle.
"""
import numpy as np
import pytest

import workloads as W
from tests.ulp import compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402
from paper_2001_09258_amd import autograd as A  # noqa: E402

UNARY = ["sin", "cos", "tan", "exp", "log", "tanh"]
BOUND1, BOUND2 = 2.5, 4.0
NPD = {"f64": np.float64, "f32": np.float32}


@pytest.fixture(scope="session", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()


def _grads(fn, dt, n, seed):
    rng = np.random.default_rng(seed)
    x = W.autograd_inputs(fn, n, seed).astype(NPD[dt])
    y = W.autograd_inputs(fn, n, seed + 1).astype(NPD[dt])
    g = rng.standard_normal(n).astype(NPD[dt])
    return x, y, g


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("fn", UNARY)
def test_unary_backward_vs_oracle(fn, dt):
    import oracle.batch as OB
    n = 8192 + 37
    x, _, g = _grads(fn, dt, n, 11)
    print("bwd", fn, dt, flush=True)
    tx, tg = torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda()
    (gx,) = L.backward(fn, (tx,), tg)
    got = gx.cpu().numpy().astype(np.float64)
    ((rn, hi, lo),) = OB.evaluate_grad(fn, dt, x, g)
    r = compare(got, rn, hi, lo, dt, BOUND1)
    assert r["violations"] == 0 and r["special_mismatch"] == 0, r


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("fn", ["pow", "atan2"])
def test_binary_backward_vs_oracle(fn, dt):
    import oracle.batch as OB
    n = 8192 + 37
    x, y, g = _grads(fn, dt, n, 21)
    print("bwd", fn, dt, flush=True)
    tx, ty, tg = (torch.from_numpy(v).cuda() for v in (x, y, g))
    g0, g1 = L.backward(fn, (tx, ty), tg)
    want = OB.evaluate_grad(fn, dt, x, g, y)
    for got, (rn, hi, lo) in zip((g0, g1), want):
        r = compare(got.cpu().numpy().astype(np.float64), rn, hi, lo, dt, BOUND2)
        assert r["violations"] == 0 and r["special_mismatch"] == 0, r


FNS = {"sin": A.sin, "cos": A.cos, "tan": A.tan, "exp": A.exp, "log": A.log, "tanh": A.tanh}


@pytest.mark.parametrize("fn", UNARY)
def test_autograd_matches_central_differences(fn):
    n = 4096
    x0 = torch.from_numpy(W.autograd_inputs(fn, n, 3).astype(np.float64)).cuda()
    if fn == "tan":
        x0 = x0 * 0.1                     # stay clear of the poles
    x = x0.clone().requires_grad_(True)
    y = FNS[fn](x)
    g = torch.ones_like(y)
    y.backward(g)
    h = 1e-6 * torch.clamp(x0.abs(), min=1.0)
    fp, fm = L.evaluate(fn, x0 + h), L.evaluate(fn, x0 - h)
    fd = (fp - fm) / (2 * h)
    # truncation error O(h^2) plus the rounding noise of the difference itself
    tol = 1e-6 * fd.abs() + 4 * 2.0 ** -52 * torch.maximum(fp.abs(), fm.abs()) / h
    bad = ((x.grad - fd).abs() > tol).sum().item()
    assert bad == 0, ((x.grad - fd).abs() / tol).max().item()


def test_binary_autograd_matches_central_differences():
    n = 4096
    a = torch.from_numpy(W.autograd_inputs("pow", n, 5).astype(np.float64)).cuda()
    b = torch.from_numpy(W.autograd_inputs("pow", n, 6).astype(np.float64)).cuda() * 0.3
    for fn, F in (("pow", A.pow), ("atan2", A.atan2)):
        xa = a.clone().requires_grad_(True)
        xb = b.clone().requires_grad_(True)
        F(xa, xb).backward(torch.ones_like(a))
        ha = 1e-6 * a.abs().clamp(min=1.0)
        hb = 1e-6 * b.abs().clamp(min=1.0)
        pa, ma = L.evaluate(fn, a + ha, b), L.evaluate(fn, a - ha, b)
        pb, mb = L.evaluate(fn, a, b + hb), L.evaluate(fn, a, b - hb)
        fda, fdb = (pa - ma) / (2 * ha), (pb - mb) / (2 * hb)
        for got, fd, p, m, h in ((xa.grad, fda, pa, ma, ha), (xb.grad, fdb, pb, mb, hb)):
            tol = 1e-6 * fd.abs() + 4 * 2.0 ** -52 * torch.maximum(p.abs(), m.abs()) / h
            assert ((got - fd).abs() > tol).sum().item() == 0, fn


def test_gradcheck_float64():
    x = (torch.rand(24, dtype=torch.float64, device="cuda") * 2 + 0.2).requires_grad_(True)
    xt = (torch.rand(24, dtype=torch.float64, device="cuda") * 1.2 + 0.1).requires_grad_(True)
    for fn, F in FNS.items():
        arg = xt if fn == "tan" else x            # keep tan away from its pole at pi/2
        assert torch.autograd.gradcheck(F, (arg,), eps=1e-6, atol=1e-9, rtol=1e-7), fn
    y = (torch.rand(24, dtype=torch.float64, device="cuda") * 2 + 0.2).requires_grad_(True)
    assert torch.autograd.gradcheck(A.pow, (x, y), eps=1e-6, atol=1e-9, rtol=1e-7)
    assert torch.autograd.gradcheck(A.atan2, (y, x), eps=1e-6, atol=1e-9, rtol=1e-7)


@pytest.mark.parametrize("fn", ["sin", "exp", "log", "tanh", "pow", "atan2"])
def test_autograd_full_size(fn):
    """Forward + backward on 2^24 binary32 elements x ~ U[0.1, 10]; 4096
    sampled gradients against the oracle."""
    import oracle.batch as OB
    n = 1 << 24
    x = W.autograd_inputs(fn, n, 0)
    y = W.autograd_inputs(fn, n, 1)
    tx = torch.from_numpy(x).cuda().requires_grad_(True)
    ty = torch.from_numpy(y).cuda().requires_grad_(True)
    print("autograd full size", fn, flush=True)
    out = {"pow": lambda: A.pow(tx, ty), "atan2": lambda: A.atan2(tx, ty)}.get(
        fn, lambda: {"sin": A.sin, "exp": A.exp, "log": A.log, "tanh": A.tanh}[fn](tx))()
    out.backward(torch.ones_like(out))
    torch.cuda.synchronize()
    idx = np.random.default_rng(1).integers(0, n, 4096)
    g = np.ones(idx.size)
    if fn in ("pow", "atan2"):
        want = OB.evaluate_grad(fn, "f32", x[idx], g, y[idx])
        got = (tx.grad.cpu().numpy()[idx], ty.grad.cpu().numpy()[idx])
        bound = BOUND2
    else:
        want = OB.evaluate_grad(fn, "f32", x[idx], g)
        got = (tx.grad.cpu().numpy()[idx],)
        bound = BOUND1
    for gv, (rn, hi, lo) in zip(got, want):
        r = compare(gv.astype(np.float64), rn, hi, lo, "f32", bound)
        assert r["violations"] == 0 and r["special_mismatch"] == 0, r


# ---------------------------------------------------------------------------
# backward kernels away from U[0.1, 10]
# ---------------------------------------------------------------------------
def _run_bwd(fn, dt, a, b, g):
    ins = [torch.from_numpy(np.ascontiguousarray(v).astype(NPD[dt])).cuda()
           for v in ((a,) if b is None else (a, b))]
    outs = L.backward(fn, ins, torch.from_numpy(g.astype(NPD[dt])).cuda())
    return [o.cpu().numpy().astype(np.float64) for o in outs]


def _check_grad(got, want, dt, bound, what):
    rn, hi, lo = want
    r = compare(got, rn, hi, lo, dt, bound, subnormal="report")
    if r["subnormal_mismatch"]:
        print("%s: %d of %d subnormal gradients not correctly rounded"
              % (what, r["subnormal_mismatch"], r["subnormal_results"]), flush=True)
    assert r["violations"] == 0 and r["special_mismatch"] == 0, (what, r)


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_pow_backward_whole_range_vs_oracle(dt):
    """pow partials with |y log x| out to the overflow and underflow edges
    (gradients rounded once, also into subnormals and at overflow), and
    x < 0 with integer y: d/dx = y (-1)^(y-1) |x|^(y-1), d/dy = NaN."""
    import oracle.batch as OB
    n = 6000
    a, b, g = W.backward_edges("pow", dt, n, 0)
    print("bwd edges pow", dt, flush=True)
    gx, gy = _run_bwd("pow", dt, a, b, g)
    a64, b64, g64 = (v.astype(np.float64) for v in (a, b, g))
    wx, wy = OB.evaluate_grad("pow", dt, np.abs(a64), g64, b64)
    neg = a64 < 0
    flip = neg & (np.fmod(b64, 2.0) == 0)                 # y even: y - 1 odd
    wx = tuple(np.where(flip, -v, v) for v in wx)
    _check_grad(gx, wx, dt, BOUND2, "pow d/dx")
    _check_grad(gy[~neg], tuple(v[~neg] for v in wy), dt, BOUND2, "pow d/dy")
    assert np.isnan(gy[neg]).all()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_atan2_backward_extreme_magnitudes_vs_oracle(dt):
    """atan2 partials with y, x near overflow and underflow (the common
    power-of-two prescaling keeps x^2 + y^2 finite)."""
    import oracle.batch as OB
    a, b, g = W.backward_edges("atan2", dt, 6000, 0)
    print("bwd edges atan2", dt, flush=True)
    gy, gx = _run_bwd("atan2", dt, a, b, g)
    wy, wx = OB.evaluate_grad("atan2", dt, a.astype(np.float64), g.astype(np.float64),
                              b.astype(np.float64))
    _check_grad(gy, wy, dt, BOUND2, "atan2 d/dy")
    _check_grad(gx, wx, dt, BOUND2, "atan2 d/dx")


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_tanh_backward_large_arguments_vs_oracle(dt):
    """tanh' = 1/cosh^2 out to where it underflows (|x| up to 380 binary64,
    60 binary32): no 1 - tanh^2 cancellation, gradual underflow."""
    import oracle.batch as OB
    a, _, g = W.backward_edges("tanh", dt, 6000, 0)
    print("bwd edges tanh", dt, flush=True)
    (gx,) = _run_bwd("tanh", dt, a, None, g)
    (want,) = OB.evaluate_grad("tanh", dt, a.astype(np.float64), g.astype(np.float64))
    _check_grad(gx, want, dt, BOUND1, "tanh'")


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_tan_backward_near_poles_vs_oracle(dt):
    """tan' = 1 + tan^2 at the floating-point numbers next to multiples of
    pi/2 (the odd ones are the poles, where tan' reaches ~2^106)."""
    import oracle.batch as OB
    from tests.trig_hard_cases import near_multiples
    x = near_multiples(dt)
    x = x[::max(1, x.size // 6000)]
    g = np.random.default_rng(9).standard_normal(x.size)
    x, g = x.astype(NPD[dt]), g.astype(NPD[dt])
    print("bwd edges tan", dt, x.size, flush=True)
    (gx,) = _run_bwd("tan", dt, x, None, g)
    (want,) = OB.evaluate_grad("tan", dt, x.astype(np.float64), g.astype(np.float64))
    _check_grad(gx, want, dt, BOUND1, "tan'")


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_backward_special_points(dt):
    """The values the header documents: pow at x = +-0 (d/dx = g y
    pow(x, y - 1) with Annex F pow; d/dy = 0 for y >= 0, NaN for y < 0), at
    x < 0 with non-integer y (both NaN), at x = 1 (d/dy = 0) and y = 0
    (d/dx = 0); atan2 at (0, 0) (both NaN) and on the axes."""
    import math
    xs = [0.0, -0.0, 0.0, -0.0, 0.0, 0.0, -0.0, 0.0, -2.0, 1.0, 3.0]
    ys = [2.0, 2.0, 3.0, 3.0, 1.0, 0.5, -1.0, 0.0, 0.5, 7.0, 0.0]
    g = 1.5
    gx, gy = _run_bwd("pow", dt, np.array(xs), np.array(ys), np.full(len(xs), g))
    for i, (x, y) in enumerate(zip(xs, ys)):
        if x < 0 and y != math.floor(y):
            assert math.isnan(gx[i]) and math.isnan(gy[i]), (x, y)
            continue
        if x == 0.0:
            with np.errstate(divide="ignore"):
                p = float(np.power(np.float64(x), np.float64(y - 1.0)))   # C99 Annex F pow
            wx = 0.0 if y == 0 else g * (y * p)
            wy = 0.0 if y >= 0 else float("nan")
            assert (gx[i] == wx and math.copysign(1, gx[i]) == math.copysign(1, wx)), (x, y, gx[i], wx)
            assert (math.isnan(wy) and math.isnan(gy[i])) or gy[i] == wy, (x, y, gy[i], wy)
        if x == 1.0:
            assert gy[i] == 0.0, (x, y, gy[i])
        if y == 0.0:
            assert gx[i] == 0.0, (x, y, gx[i])
    ay = np.array([0.0, 0.0, 3.0, -2.0])
    ax = np.array([0.0, -2.0, 0.0, 0.0])
    gyy, gxx = _run_bwd("atan2", dt, ay, ax, np.full(4, g))
    assert np.isnan(gyy[0]) and np.isnan(gxx[0])
    assert gyy[1] == g * -0.5 and gxx[1] == 0.0              # d/dy = x / x^2 = 1/x
    assert gyy[2] == 0.0 and gxx[2] == -g / 3.0
    assert gyy[3] == 0.0 and gxx[3] == g / 2.0
