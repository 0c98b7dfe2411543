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
