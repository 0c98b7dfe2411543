"""Exhaustive sweeps over every binary32 bit pattern for sin, cos, tan, exp,
exp2, log, log2, sinh, cosh, tanh, asin, acos, atan, log10, log1p, exp10,
expm1, cbrt, asinh, acosh, atanh, erf, erfc, lgamma and tgamma (test infrastructure;
minutes per function, so run by hand).

    python -m tests.sweep32 libm [--fns sin,exp,log,...] [--threads N]
        the oracle's fast stage against the host libm's binary64 result
        rounded to binary32, all 2^32 inputs: where the two differ, the
        binary64 value must lie within two of its ulps of a binary32
        midpoint (a double rounding); every differing and every undecided
        input is re-evaluated by the ball oracle.
    python -m tests.sweep32 gpu [--fns ...] [--variants u10,u35] [--threads N] [--via-f64]
        the GPU entry points on all 2^32 inputs against the oracle (ULP
        metric of tests/ulp.py; NaN, inf, zero and subnormal results
        bit-exact; with --via-f64 the binary32-through-binary64 forms, whose
        subnormal results round twice and are counted as mismatches).
Each prints one JSON line per function (and variant).
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import fast32  # noqa: E402

TOTAL = 1 << 32
CHUNK = 1 << 22


def _ball_confirm(fn, bits, limit=4096):
    """Ball-oracle results for up to ``limit`` inputs, and whether they equal
    the fast stage's."""
    import oracle
    bits = np.asarray(bits, np.uint32)[:limit]
    if bits.size == 0:
        return 0, 0
    x = bits.view(np.float32)
    rn_b = oracle.evaluate(fn, "f32", x.astype(np.float64))[0]
    rn_f, _, _, und = fast32.fast_eval(fn, x)
    ok = (rn_b == rn_f.astype(np.float64)) | (np.isnan(rn_b) & np.isnan(rn_f))
    ok |= und                       # undecided: the ball result stands
    return int(bits.size), int((~ok).sum())


def sweep_libm(fn, threads, total=TOTAL, start0=0):
    fast32.load()
    t0 = time.time()
    agg = dict(n=0, undecided=0, differ=0, differ_explained=0)
    differ, undec = [], []
    with cf.ThreadPoolExecutor(threads) as ex:
        futs = [ex.submit(fast32.sweep_libm, fn, start0 + s, min(CHUNK, total - s), 1 << 12)
                for s in range(0, total, CHUNK)]
        for f in futs:
            st, d, u = f.result()
            for k in agg:
                agg[k] += getattr(st, k)
            differ.append(d)
            undec.append(u)
    differ = np.concatenate(differ) if differ else np.zeros(0, np.uint32)
    undec = np.concatenate(undec) if undec else np.zeros(0, np.uint32)
    nd, bad_d = _ball_confirm(fn, differ)
    nu, _ = _ball_confirm(fn, undec)
    agg.update(fn=fn, seconds=round(time.time() - t0, 1), threads=threads,
               differ_checked_by_ball=nd, differ_ball_disagrees_with_fast=bad_d,
               undecided_resolved_by_ball=nu)
    return agg


def sweep_gpu(fn, variant, threads, total=TOTAL, gpu_chunk=1 << 26, via_f64=False):
    import torch
    import paper_2001_09258_amd as L
    L.load()
    fast32.load()
    bound = 1.0 if variant == "u10" else 3.5
    t0 = time.time()
    agg = dict(n=0, undecided=0, special_mismatch=0, violations=0, n_reg=0)
    max_ulp, sum_ulp, worst = 0.0, 0.0, 0
    bad_all, und_all = [], []
    with cf.ThreadPoolExecutor(threads) as ex:
        pending = []
        for g0 in range(0, total, gpu_chunk):
            n = min(gpu_chunk, total - g0)
            xb = torch.arange(g0, g0 + n, dtype=torch.int64, device="cuda")
            xb = torch.where(xb >= (1 << 31), xb - (1 << 32), xb).to(torch.int32)
            x = xb.view(torch.float32)
            y = L.evaluate(fn, x, variant=variant, via_f64=via_f64)
            yh = y.cpu().numpy()
            del xb, x, y
            for s in range(0, n, CHUNK):
                c = min(CHUNK, n - s)
                pending.append(ex.submit(fast32.check, fn, g0 + s, c, yh[s:s + c], bound, 1 << 10))
            print("  %s %s: GPU chunk %d/%d queued" % (fn, variant, g0 // gpu_chunk + 1,
                                                      (total + gpu_chunk - 1) // gpu_chunk),
                  file=sys.stderr, flush=True)
            # keep the host memory bounded: wait for all but the last chunk's checks
            done = [p for p in pending[:-(gpu_chunk // CHUNK)]]
            for p in done:
                st, b, u = p.result()
                for k in agg:
                    agg[k] += getattr(st, k)
                sum_ulp += st.sum_ulp
                if st.max_ulp > max_ulp:
                    max_ulp, worst = st.max_ulp, st.worst
                bad_all.append(b)
                und_all.append(u)
            pending = pending[len(done):]
        for p in pending:
            st, b, u = p.result()
            for k in agg:
                agg[k] += getattr(st, k)
            sum_ulp += st.sum_ulp
            if st.max_ulp > max_ulp:
                max_ulp, worst = st.max_ulp, st.worst
            bad_all.append(b)
            und_all.append(u)
    agg.update(fn=fn, variant=variant + ("_via_f64" if via_f64 else ""), max_ulp=round(max_ulp, 4),
               mean_ulp=round(sum_ulp / max(agg["n_reg"], 1), 4),
               worst_input=float(np.uint32(worst).view(np.float32)),
               bad_inputs=[float(v) for v in np.concatenate(bad_all)[:8].view(np.float32)] if bad_all else [],
               seconds=round(time.time() - t0, 1), threads=threads)
    return agg


def main():
    p = argparse.ArgumentParser()
    p.add_argument("mode", choices=["libm", "gpu"])
    p.add_argument("--fns", default="sin,exp,log")
    p.add_argument("--variants", default="u10")
    p.add_argument("--threads", type=int, default=min(16, os.cpu_count() or 4))
    p.add_argument("--total", type=int, default=TOTAL, help="inputs from bit pattern 0 (testing)")
    p.add_argument("--via-f64", action="store_true",
                   help="the binary32-through-binary64 entry points (u10 names)")
    a = p.parse_args()
    for fn in a.fns.split(","):
        if a.mode == "libm":
            print(json.dumps(sweep_libm(fn, a.threads, a.total)), flush=True)
        else:
            for v in a.variants.split(","):
                print(json.dumps(sweep_gpu(fn, v, a.threads, a.total, via_f64=a.via_f64)),
                      flush=True)


if __name__ == "__main__":
    main()
