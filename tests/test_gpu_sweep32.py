"""The GPU binary32 sin, cos, tan, exp, exp2, log, log2, sinh, cosh, tanh,
asin, acos, atan, log10, log1p, exp10, expm1, cbrt, asinh, acosh, atanh,
erf, erfc, lgamma and tgamma against the oracle's fast stage on 8 stretches of 2^20 consecutive bit
patterns spread over all 2^32 (the full sweep over every pattern is
tests/sweep32.py, run by hand): every result within its bound, NaN, inf,
zero and subnormal results bit-exact."""
import numpy as np
import pytest

from oracle import fast32

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402

STARTS = [(i << 29) + ((i * 0x9e3779b) & 0x1fff0000) for i in range(8)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    fast32.load()


KINDS = [(f, "u10") for f in ("sin", "cos", "tan", "exp", "exp2", "log", "log2", "sinh", "cosh",
                               "tanh", "asin", "acos", "atan", "log10", "log1p", "exp10", "expm1",
                               "cbrt", "asinh", "acosh", "atanh", "erf", "erfc", "lgamma", "tgamma")]
KINDS += [(f, "u35") for f in ("sin", "cos", "tan", "asin", "acos", "atan", "log", "sinh", "cosh",
                                "tanh")]


@pytest.mark.parametrize("fn,variant", KINDS)
def test_stretches_against_the_oracle(fn, variant):
    bound = 1.0 if variant == "u10" else 3.5
    n = 1 << 20
    print("sweep", fn, variant, flush=True)
    worst = 0.0
    for s in STARTS:
        bits = np.arange(s, s + n, dtype=np.uint64).astype(np.uint32)
        x = torch.from_numpy(bits.view(np.float32)).cuda()
        y = L.evaluate(fn, x, variant=variant).cpu().numpy()
        st, bad, und = fast32.check(fn, s, n, y, bound)
        assert st.violations == 0 and st.special_mismatch == 0, \
            (fn, variant, hex(s), bad[:4].view(np.float32))
        worst = max(worst, st.max_ulp)
    print("  max ulp %.4f" % worst, flush=True)
