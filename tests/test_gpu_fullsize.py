"""Full benchmark size, in the launch shape the benchmark times.

Every kernel of the benchmark step (15 function-variants x {binary64,
binary32} on the 2^26-element mixture) and of the large-argument workload
(sin, cos, tan u10/u35, fmod, remainder x {binary64, binary32} on 2^26
elements) runs on its full-size input after the launch-shape tuner has
picked its shape on those buffers, exactly as the benchmark does; 2^16
sampled outputs plus the first and last are checked against the oracle one
by one (ULP bound, special classes and binary64/binary32 subnormal results
bit-exact; exact functions bit-exact), and then every output of every
kernel: through the oracle's fast stages (sin, cos, tan, exp, exp2, log,
log2, sinh, cosh, tanh, pow, atan2; the inputs they cannot decide through
the ball oracle), and bit-exact against the host's fmod and the exact
array remainder.
"""
import concurrent.futures as cf

import numpy as np
import pytest

import workloads as W
from tests.exact_ref import fmod as exact_fmod, ieee_remainder
from tests.gpu_common import check_values, to_device, to_host

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2001_09258_amd as L  # noqa: E402
from oracle import fast32, fast64  # noqa: E402

N = 1 << 26
SAMPLES = 1 << 16
FAST_FNS = set(fast32.FNS) | set(fast32.FNS2)
STEP = [("sin", "u10"), ("sin", "u35"), ("cos", "u10"), ("cos", "u35"), ("tan", "u10"),
        ("tan", "u35"), ("exp", "u10"), ("exp2", "u10"), ("log", "u10"), ("log2", "u10"),
        ("pow", "u10"), ("atan2", "u10"), ("sinh", "u10"), ("cosh", "u10"), ("tanh", "u10")]
LARGE = [("sin", "u10"), ("sin", "u35"), ("cos", "u10"), ("cos", "u35"), ("tan", "u10"),
         ("tan", "u35"), ("fmod", "exact"), ("remainder", "exact")]
CASES = [("mixture", fn, v, dt) for dt in ("f64", "f32") for fn, v in STEP]
CASES += [("large_args", fn, v, dt) for dt in ("f64", "f32") for fn, v in LARGE]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    yield
    L.tune_reset()


@pytest.mark.parametrize("workload,fn,variant,dt", CASES, ids=["-".join(c) for c in CASES])
def test_full_size_tuned_sampled(workload, fn, variant, dt):
    gen = W.mixture if workload == "mixture" else W.large_args
    binary = fn in L.BINARY
    with cf.ThreadPoolExecutor(2) as ex:
        fa = ex.submit(gen, fn, dt, N, 0)
        fb = ex.submit(gen, fn, dt, N, 1) if binary else None
        a, b = fa.result(), (fb.result() if fb else None)
    print("full size tuned", workload, fn, variant, dt, flush=True)
    ta = to_device(a, dt)
    tb = to_device(b, dt) if binary else None
    out = torch.empty_like(ta)
    shape = L.tune(fn, ta, tb, variant=variant, out=out)
    L.evaluate(fn, ta, tb, variant=variant, out=out)
    idx = np.random.default_rng(17).integers(0, N, SAMPLES)
    idx = np.unique(np.concatenate([idx, [0, N - 1]]))
    y = to_host(out[torch.from_numpy(idx).cuda()])
    torch.cuda.synchronize()
    res = check_values(fn, variant, dt, a[idx], None if b is None else b[idx], y,
                       label="full size %s %s" % (workload, shape))
    print("  shape %s: %d checked, max %.3f ulp" % (shape, idx.size, res["max_ulp"]), flush=True)
    # every output: the oracle's fast stage for the unary functions it
    # covers (its undecided inputs through the ball oracle), the host's
    # exact fmod and the exact array remainder for the exact functions
    if fn in FAST_FNS or fn in ("fmod", "remainder"):
        y_all = to_host(out)
        torch.cuda.synchronize()
        if fn in ("fmod", "remainder"):
            want = exact_fmod(a, b) if fn == "fmod" else ieee_remainder(a, b).astype(a.dtype)
            same = (y_all == want) | (np.isnan(y_all) & np.isnan(want))
            same &= (np.signbit(y_all) == np.signbit(want)) | np.isnan(want)
            assert same.all(), (a[~same][:3], b[~same][:3], y_all[~same][:3])
            print("  all %d outputs bit-exact" % N, flush=True)
            return
        fast = fast64 if dt == "f64" else fast32
        bound = 1.0 if variant == "u10" else 3.5
        tot = fast.check_all(fn, a, y_all, bound, z=b)
        if tot["undecided"]:
            u = tot["undecided_idx"]
            assert tot["undecided"] == u.size, "more undecided inputs than listed"
            check_values(fn, variant, dt, a[u], None if b is None else b[u], y_all[u],
                         label="full size, undecided")
        assert tot["violations"] == 0 and tot["special_mismatch"] == 0, \
            (fn, variant, dt, a[tot["bad"][:4]], y_all[tot["bad"][:4]])
        print("  all %d outputs: max %.4f ulp, mean %.4f, %d by the ball oracle"
              % (N, tot["max_ulp"], tot["sum_ulp"] / max(tot["n_reg"], 1), tot["undecided"]),
              flush=True)
