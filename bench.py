#!/usr/bin/env python3
"""Benchmark of the libm_hip hot path on one MI355X.

One step = one pass of the full function set over one batch of synthetic
input: sin/cos/tan (u10 and u35), exp, exp2, log, log2, pow, atan2, sinh,
cosh, tanh (u10), in binary64 and binary32, 2^26 elements each (30 kernel
launches; the mixture of 49% U[-1e4, 1e4], 50% log-uniform magnitudes, 1%
special values).  Inputs are resident in HBM before timing starts.

Prints one JSON line: whole-step throughput in Gelem/s, the roofline of the
dominant kernel (its own average duration measured with HIP events on the
launch stream), per-function throughput, and the CPU oracle's rate on a
bounded sample of the same inputs.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12           # bytes/s, MI355X HBM3E
FP64_PEAK = 78.6e12         # flop/s, dense vector FP64
FP32_PEAK = 157.3e12        # flop/s, vector FP32 (packed)

FUNCS = [("sin", "u10"), ("sin", "u35"), ("cos", "u10"), ("cos", "u35"),
         ("tan", "u10"), ("tan", "u35"), ("exp", "u10"), ("exp2", "u10"),
         ("log", "u10"), ("log2", "u10"), ("pow", "u10"), ("atan2", "u10"),
         ("sinh", "u10"), ("cosh", "u10"), ("tanh", "u10")]
BINARY = ("pow", "atan2")
ESIZE = {"f64": 8, "f32": 4}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--n", type=int, default=1 << 26)
    p.add_argument("--reps", type=int, default=3, help="per-kernel timing repeats")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=2048,
                   help="oracle sample per (function, dtype)")
    p.add_argument("--only", default="", help="comma list fn:var:dt to restrict the step")
    return p.parse_args()


def make_plan(only):
    plan = [(fn, v, dt) for dt in ("f64", "f32") for fn, v in FUNCS]
    if only:
        keep = set(tuple(s.split(":")) for s in only.split(","))
        plan = [p for p in plan if p in keep]
    return plan


def gen_inputs(plan, n):
    import workloads as W

    def one(item):
        fn, v, dt = item
        a = W.config2(fn, dt, n, 0)
        b = W.config2(fn, dt, n, 1) if fn in BINARY else None
        return item, a, b

    out = {}
    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        for item, a, b in ex.map(one, plan):
            out[item] = (a, b)
    return out


def cpu_baseline(inputs, sample):
    """The oracle as it stands, on the first ``sample`` elements of every
    (function, dtype) input of the step, over a process pool on all cores."""
    import oracle
    from oracle.batch import default_workers
    workers = default_workers()
    total = 0
    t0 = time.perf_counter()
    for (fn, v, dt), (a, b) in inputs.items():
        oracle.evaluate(fn, dt, a[:sample], None if b is None else b[:sample], workers=workers)
        total += min(sample, a.shape[0])
    dt_s = time.perf_counter() - t0
    return {"value": total / dt_s / 1e9, "unit": "Gelem/s", "cores": workers,
            "kind": "oracle",
            "sample": "first %d elements of each of the %d (function, dtype) inputs of the "
                      "step (%d elements, %.1f s)" % (sample, len(inputs), total, dt_s)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the method is elementwise; "
              "see the sharding notes in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2001_09258_amd as L

    lib = L.load()
    plan = make_plan(args.only)
    n = args.n
    t_gen = time.perf_counter()
    host = gen_inputs(plan, n)
    print("bench: generated %d input sets of %d elements in %.1f s"
          % (len(plan), n, time.perf_counter() - t_gen), file=sys.stderr, flush=True)

    dev = {}
    for item in plan:
        fn, v, dt = item
        a, b = host[item]
        ta = torch.from_numpy(a).cuda()
        tb = torch.from_numpy(b).cuda() if b is not None else None
        dev[item] = (ta, tb, torch.empty_like(ta))
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    calls = []
    for item in plan:
        fn, v, dt = item
        ta, tb, to = dev[item]
        f = getattr(lib, L.entry_name(fn, v, dt))
        if tb is None:
            calls.append((item, f, (ta.data_ptr(), to.data_ptr(), n, sh)))
        else:
            calls.append((item, f, (ta.data_ptr(), tb.data_ptr(), to.data_ptr(), n, sh)))

    def step():
        for item, f, cargs in calls:
            st = f(*cargs)
            if st != 0:
                raise RuntimeError("%s: %s" % (item, lib.libm_hip_last_error()))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    elems = n * len(plan)
    value = elems / (ms_step * 1e-3) / 1e9
    print("bench: %.3f ms per step" % ms_step, file=sys.stderr, flush=True)

    # per-kernel durations: HIP events on the launch stream around each call
    per = {}
    for item, f, cargs in calls:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.reps):
            f(*cargs)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.reps
        fn, v, dt = item
        nb = ESIZE[dt] * (3 if fn in BINARY else 2)
        per["%s_%s_%s" % item] = {"ms": round(ms, 4), "gelem_s": round(n / ms / 1e6, 2),
                                  "hbm_frac": round(nb * n / (ms * 1e-3) / HBM_PEAK, 4)}
    dom = max(per, key=lambda k: per[k]["ms"])
    fn, v, dt = dom.split("_")
    nb = ESIZE[dt] * (3 if fn in BINARY else 2)
    dom_ms = per[dom]["ms"]
    achieved = nb * n / (dom_ms * 1e-3)
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(achieved / 1e9, 1),
                "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK, 4), "traffic": None,
                "algorithmic_bytes_per_elem": nb, "elements_per_launch": n,
                "avg_launch_ms": dom_ms}

    result = {"metric": "Gelem/s per function at <=1.0/3.5 ULP; % of HBM or VALU roofline",
              "value": round(value, 3), "unit": "Gelem/s", "n_gpus": 1,
              "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "dtype": "f64+f32", "data": "synthetic",
              "config": {"workload": "full FP64+FP32 function set (15 function-variants x 2 "
                                     "dtypes) on 2^26 elements each, config-2 mixture",
                         "elements_per_step": elems, "functions": len(plan),
                         "parallelism": "single GPU"},
              "roofline": roofline, "per_function": per}
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(host, args.cpu_sample)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
