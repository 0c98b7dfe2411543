"""Random binary64 bit patterns through the GPU entry points against the
oracle's binary64 fast stage (test infrastructure; minutes per run, so run
by hand).  The patterns are uniform over all 2^64 (every sign, exponent and
special class in proportion; two independent arrays for pow and atan2),
seeded per function.

    python -m tests.sweep64 [--fns sin,exp,...] [--count N] [--threads N]
        every variant of each function; one JSON line per function and
        variant (ULP metric of tests/ulp.py; NaN, inf, zero and subnormal
        results bit-exact; undecided inputs through the ball oracle).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import fast64  # noqa: E402


def sweep(fn, variant, count, threads, chunk=1 << 24):
    import torch
    import paper_2001_09258_amd as L
    from tests.gpu_common import check_values
    L.load()
    fast64.load()
    bound = 1.0 if variant == "u10" else 3.5
    binary = fn in L.BINARY
    rng = np.random.default_rng(sum(map(ord, fn)) * 7 + len(variant))
    t0 = time.time()
    agg = dict(n=0, undecided=0, special_mismatch=0, violations=0, n_reg=0)
    max_ulp, sum_ulp, bad = 0.0, 0.0, []
    for s in range(0, count, chunk):
        n = min(chunk, count - s)
        a = rng.integers(0, 1 << 64, n, dtype=np.uint64).view(np.float64)
        b = rng.integers(0, 1 << 64, n, dtype=np.uint64).view(np.float64) if binary else None
        ta = torch.from_numpy(a).cuda()
        tb = torch.from_numpy(b).cuda() if binary else None
        y = L.evaluate(fn, ta, tb, variant=variant).cpu().numpy()
        tot = fast64.check_all(fn, a, y, bound, threads=threads, z=b)
        if tot["undecided"]:
            u = tot["undecided_idx"]
            assert tot["undecided"] == u.size, "more undecided inputs than listed"
            check_values(fn, variant, "f64", a[u], None if b is None else b[u], y[u],
                         label="sweep64, undecided")
        for k in agg:
            agg[k] += tot[k]
        sum_ulp += tot["sum_ulp"]
        max_ulp = max(max_ulp, tot["max_ulp"])
        bad += [float(v) for v in a[tot["bad"][:4]]]
        print("  %s %s: %d / %d" % (fn, variant, s + n, count), file=sys.stderr, flush=True)
    agg.update(fn=fn, variant=variant, max_ulp=round(max_ulp, 4),
               mean_ulp=round(sum_ulp / max(agg["n_reg"], 1), 4), bad_inputs=bad[:8],
               seconds=round(time.time() - t0, 1))
    return agg


def main():
    import paper_2001_09258_amd as L
    p = argparse.ArgumentParser()
    p.add_argument("--fns", default=",".join(sorted(set(fast64.FNS) | set(fast64.FNS2))))
    p.add_argument("--count", type=int, default=1 << 26)
    p.add_argument("--threads", type=int, default=min(16, os.cpu_count() or 4))
    a = p.parse_args()
    for fn in a.fns.split(","):
        for v in L.VARIANTS[fn]:
            if L.served(fn, v, "f64"):
                print(json.dumps(sweep(fn, v, a.count, a.threads)), flush=True)


if __name__ == "__main__":
    main()
