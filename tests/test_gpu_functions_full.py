"""Every function that the oracle's fast stages cover, in every variant and
in binary64 and binary32, on 2^24 elements of the benchmark's input for that
function (workloads.function_mixture; two operands for pow and atan2): every
output is checked against the oracle (tests/ulp.py's metric; NaN, inf, zero
and subnormal results bit-exact), the inputs the fast stages cannot decide
through the ball oracle."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import check_values, to_device, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402
from oracle import fast32, fast64  # noqa: E402

N = 1 << 24
FNS = sorted(set(fast64.FNS) | set(fast64.FNS2))
CASES = [(fn, v, dt) for fn in FNS for v in L.VARIANTS[fn] for dt in ("f64", "f32")
         if L.served(fn, v, dt)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    fast32.load()
    fast64.load()


@pytest.mark.parametrize("fn,variant,dt", CASES, ids=["-".join(c) for c in CASES])
def test_every_output_against_the_oracle(fn, variant, dt):
    binary = fn in L.BINARY
    a = W.function_mixture(fn, dt, N, 70)
    b = W.function_mixture(fn, dt, N, 71) if binary else None
    print("all outputs", fn, variant, dt, flush=True)
    ta = to_device(a, dt)
    tb = to_device(b, dt) if binary else None
    y = to_host(L.evaluate(fn, ta, tb, variant=variant))
    torch.cuda.synchronize()
    fast = fast64 if dt == "f64" else fast32
    bound = 1.0 if variant == "u10" else 3.5
    tot = fast.check_all(fn, a, y, bound, z=b)
    if tot["undecided"]:
        u = tot["undecided_idx"]
        assert tot["undecided"] == u.size, "more undecided inputs than listed"
        check_values(fn, variant, dt, a[u], None if b is None else b[u], y[u],
                     label="all outputs, undecided")
    bad = tot["bad"][:4]
    assert tot["violations"] == 0 and tot["special_mismatch"] == 0, \
        (fn, variant, dt, a[bad], None if b is None else b[bad], y[bad])
    print("  %d outputs: max %.4f ulp, %d by the ball oracle"
          % (N, tot["max_ulp"], tot["undecided"]), flush=True)
