"""Results in the subnormal range, on the GPU entry points.

Binary64 and binary32: every result whose correctly rounded value is
subnormal must equal it bit for bit (the strict reading of the paper's
special-number handling, Section 5, "Handling of Special Numbers"); the
arguments come from workloads.subnormal_results (exp/exp2/exp10/erfc
intervals where the result underflows gradually, pow with y log2 x in the
subnormal exponent range plus exact ties, atan2 quotients and hypot pairs
of that size, subnormal arguments of the functions that return about
their argument).  bf16 and the binary32-through-binary64 form: the
subnormal mismatches are counted and reported, the ULP bound holds.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402

N = (1 << 16) + 37
CASES = [(fn, v, dt) for fn, v, dt, _ in L.all_entry_points()
         if fn in W.SUBNORMAL_FNS and dt in ("f64", "f32", "f32_via_f64", "bf16")]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()


@pytest.mark.parametrize("fn,variant,dt", CASES, ids=["-".join(c) for c in CASES])
def test_subnormal_results(fn, variant, dt):
    base = "f64" if dt == "f64" else "f32"
    a, b = W.subnormal_results(fn, base, N, 0)
    if dt == "bf16":
        a = W.round_to_bf16(a)
        b = None if b is None else W.round_to_bf16(b)
    print("subnormal results", fn, variant, dt, flush=True)
    res = check(fn, variant, dt, a, b, label="subnormal")
    if dt in ("f64", "f32"):
        assert res["subnormal_results"] > N // 3, res["subnormal_results"]
