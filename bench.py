#!/usr/bin/env python3
"""Benchmark of the libm_hip hot path on one MI355X.

One step = one pass of the full function set over one batch of synthetic
input: sin/cos/tan (u10 and u35), exp, exp2, log, log2, pow, atan2, sinh,
cosh, tanh (u10), in binary64 and binary32, 2^26 elements each (30 kernel
launches; the mixture of 49% U[-1e4, 1e4], 50% log-uniform magnitudes, 1%
special values).  Inputs are resident in HBM before timing starts.

Prints one compact JSON line on stdout (a few KB): whole-step throughput in
Gelem/s, the roofline of the dominant kernel (its own average duration,
measured with HIP events recorded on the launch stream around every launch
of the timed steps), per-kernel throughput with both roofline fractions, and
the CPU oracle's rate on a bounded sample of the same inputs.  The further
measurements (precision forms, batch, autograd, large arguments, ...) go to
stderr as they complete and, with the per-kernel details, to the file named
by ``--out``.

Rooflines.  HBM: algorithmic bytes per element (inputs read once, output
written once) against 8 TB/s.  VALU: the evaluator's vector-ALU instructions
per element, counted in the gfx950 assembly of one-element probe kernels
(``paper_2001_09258_amd/gen/valu_per_element.json``; trig functions weight
the Cody-Waite and Payne-Hanek reductions by the share of inputs each one
takes).  Issue model from the unit counts and clock (256 CUs x 4 SIMDs x 16
lanes x 2.4 GHz = 39.3 T lane-slots/s): binary64 instructions take one slot
each (the 78.6 TFLOP/s FP64 vector peak), other VALU instructions can
dual-issue and take half a slot (the 157.3 TFLOP/s FP32 peak), so an element
costs max(n_f64, n_valu / 2) slots.  The kernel's VALU peak in lane-ops/s is
39.3 T x n_valu / that cost.  A kernel's bound is the one with the larger
lower-bound time.

Before timing, every kernel's launch shape (workgroup size, packs per lane)
is autotuned on its own buffers (the library's tuner; ``--no-tune`` keeps
the defaults); the chosen shapes are part of the output.

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

HBM_PEAK = 8.0e12                       # bytes/s, MI355X HBM3E
VALU_SLOTS = 256 * 4 * 16 * 2.4e9       # VALU lane-slots/s (one binary64 lane-op each)
FP64_PEAK = 78.6e12                     # flop/s, dense vector FP64
SLOW_TRIG = {"f64": 2.0 ** 14, "f32": 65536.0}   # |x| at which trig switches to Payne-Hanek
OPS_FILE = os.path.join(ROOT, "paper_2001_09258_amd", "gen", "valu_per_element.json")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "elementwise_step_hbm_traffic.json")
CSRC = os.path.join(ROOT, "paper_2001_09258_amd", "csrc")

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
    p.add_argument("--cpu-sample", type=int, default=163840,
                   help="oracle sample per (function, dtype)")
    p.add_argument("--only", default="", help="comma list fn:var:dt to restrict the step")
    p.add_argument("--no-tune", action="store_true",
                   help="keep the default launch shapes instead of autotuning them first")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the bf16/f16/via-f64, batched and autograd measurements")
    p.add_argument("--narrow-n", type=int, default=1 << 28,
                   help="elements per bf16/f16 function")
    p.add_argument("--out", default=os.path.join("bench_results", "bench_full.json"),
                   help="file for the full result (every extra); '' to skip")
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
        a = W.mixture(fn, dt, n, 0)
        b = W.mixture(fn, dt, n, 1) if fn in BINARY else None
        return item, a, b

    out = {}
    with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 4)) as ex:
        for item, a, b in ex.map(one, plan):
            out[item] = (a, b)
    return out


def kernel_source_hash():
    """sha256 over the device code of the elementwise kernels (kernels.h, the
    evaluator headers and the generated tables), comments and blank lines
    removed; HBM traffic counters taken for other device code are not
    reported.  Host-side files (launchers, the C ABI, the tuner, the batch
    plan) do not enter it."""
    import hashlib
    import re
    h = hashlib.sha256()
    for d, _, files in sorted(os.walk(CSRC)):
        for f in sorted(files):
            if f.endswith((".h", ".inc")):
                path = os.path.join(d, f)
                with open(path) as fh:
                    text = fh.read()
                text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
                text = re.sub(r"//[^\n]*", "", text)
                code = "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())
                h.update(os.path.relpath(path, CSRC).encode())
                h.update(code.encode())
    return h.hexdigest()


def load_traffic():
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return {}
    return t.get("kernels", {}) if t.get("source_hash") == kernel_source_hash() else {}


def valu_ops(fn, v, dt, a, ops):
    """Evaluator VALU instructions per element for one input array:
    (all VALU, binary64-unit instructions, share of Payne-Hanek inputs)."""
    import numpy as np
    pre = "p64_" if dt == "f64" else "p32_"

    def get(key):
        return np.array([ops[key]["valu"], ops[key]["valu_f64"]], dtype=float)
    if fn in ("sin", "cos", "tan"):
        slow = float(np.mean(~(np.abs(a) < SLOW_TRIG[dt])))
        red = (1 - slow) * get(pre + fn + "cw") + slow * get(pre + fn + "ph")
        fin = get(pre + ("tanfin" if fn == "tan" else "sinfin") + ("35" if v == "u35" else ""))
        tot = red + fin
        return float(tot[0]), float(tot[1]), slow
    tot = get(pre + fn + ("35" if v == "u35" else ""))
    return float(tot[0]), float(tot[1]), 0.0


U10_SET = ["sin", "cos", "tan", "exp", "exp2", "log", "log2", "pow", "atan2", "sinh",
           "cosh", "tanh"]


_FLUSH = []


def time_launches(stream, fn_calls, reps):
    """Average ms of each zero-argument launcher, HIP events on ``stream``
    around every launch.  Before each timed launch a 512 MiB buffer is read
    (untimed) so that no launch finds its operands in the 256 MiB
    last-level cache left warm by the previous one; a read leaves clean
    lines, so the timed launch pays no write-back for it."""
    import torch
    if not _FLUSH:
        _FLUSH.append(torch.ones(1 << 26, dtype=torch.float64, device="cuda"))
    out = []
    for f in fn_calls:
        f()
        total = 0.0
        for _ in range(reps):
            _FLUSH[0].sum()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            f()
            e1.record(stream)
            torch.cuda.synchronize()
            total += e0.elapsed_time(e1)
        out.append(total / reps)
    return out


def checked(lib, name, f, *cargs):
    def go():
        st = f(*cargs)
        if st != 0:
            raise RuntimeError("%s: %s" % (name, lib.libm_hip_last_error()))
    return go


def extra_precision_forms(lib, L, stream, dev, n_main, n_narrow, reps):
    """The binary32 u10 set through the binary64 evaluators (2^26, binary32
    mixture) and in bf16/f16 I/O (n_narrow elements each, the mixture clamped
    to the format; one shared input per dtype and operand)."""
    import torch
    import workloads as W
    sh = stream.cuda_stream
    res = {}
    calls, names = [], []
    for fn in U10_SET:
        ta, tb, to = dev[(fn, "u10", "f32")]
        nm = L.entry_name(fn, "u10", "f32_via_f64")
        f = getattr(lib, nm)
        cargs = (ta.data_ptr(), to.data_ptr(), n_main, sh) if tb is None else \
            (ta.data_ptr(), tb.data_ptr(), to.data_ptr(), n_main, sh)
        calls.append(checked(lib, nm, f, *cargs))
        names.append(fn)
    ms = time_launches(stream, calls, reps)
    res["f32_via_f64"] = {"n": n_main, "ms_total": round(sum(ms), 4),
                          "gelem_s": round(len(ms) * n_main / sum(ms) / 1e6, 2),
                          "per_function_ms": {k: round(v, 4) for k, v in zip(names, ms)}}
    base = 1 << 26
    for dt, tdt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        ops = []
        for operand in (0, 1):
            h = W.narrow_mixture("exp", dt, base, 500 + operand)
            t = torch.from_numpy(h.astype("float32")).cuda().to(tdt)
            ops.append(t.repeat((n_narrow + base - 1) // base)[:n_narrow].contiguous())
        out = torch.empty_like(ops[0])
        calls, names = [], []
        for fn in U10_SET:
            nm = L.entry_name(fn, "u10", dt)
            f = getattr(lib, nm)
            cargs = (ops[0].data_ptr(), out.data_ptr(), n_narrow, sh) \
                if fn not in BINARY else \
                (ops[0].data_ptr(), ops[1].data_ptr(), out.data_ptr(), n_narrow, sh)
            calls.append(checked(lib, nm, f, *cargs))
            names.append(fn)
        ms = time_launches(stream, calls, reps)
        res[dt] = {"n": n_narrow, "ms_total": round(sum(ms), 4),
                   "gelem_s": round(len(ms) * n_narrow / sum(ms) / 1e6, 2),
                   "per_function_ms": {k: round(v, 4) for k, v in zip(names, ms)}}
        del ops, out
    return res


TORCH_DT = {"f64": "float64", "f32": "float32", "bf16": "bfloat16", "f16": "float16"}


def extra_batch(lib, L, stream, reps):
    """The 64-request batch: one graph-replayed persistent launch against the
    sum of the per-function launches on the same requests."""
    import torch
    import workloads as W
    sh = stream.cuda_stream
    reqs = W.batch_requests(64, 3.0, 7.0)
    tensors = []
    for fn, var, dt, n, idx in reqs:
        a, b = W.request_inputs(fn, dt, n, idx)
        tdt = getattr(torch, TORCH_DT[dt])
        ta = torch.from_numpy(a.astype("float32" if dt == "bf16" else a.dtype)).cuda().to(tdt)
        tb = None if b is None else \
            torch.from_numpy(b.astype("float32" if dt == "bf16" else b.dtype)).cuda().to(tdt)
        tensors.append((fn, var, dt, ta, tb, torch.empty_like(ta)))
    total = sum(t[3].numel() for t in tensors)
    plan = L.BatchPlan(64, use_graph=True)
    arr = (L.Request * len(tensors))()
    for i, (fn, var, dt, ta, tb, to) in enumerate(tensors):
        arr[i] = L.Request(L.FN_CODES[fn], L.VARIANT_CODES[var], L.DTYPE_CODES[dt], 0,
                           ta.data_ptr(), 0 if tb is None else tb.data_ptr(), to.data_ptr(),
                           ta.numel())

    def run_batch():
        st = plan.run_raw(arr, len(tensors), sh)
        if st != 0:
            raise RuntimeError("batch_run: %s" % lib.libm_hip_last_error())
    singles = []
    for fn, var, dt, ta, tb, to in tensors:
        nm = L.entry_name(fn, var, dt)
        f = getattr(lib, nm)
        cargs = (ta.data_ptr(), to.data_ptr(), ta.numel(), sh) if tb is None else \
            (ta.data_ptr(), tb.data_ptr(), to.data_ptr(), ta.numel(), sh)
        singles.append(checked(lib, nm, f, *cargs))

    def run_singles():
        for f in singles:
            f()
    ms_b, ms_s = time_launches(stream, [run_batch, run_singles], reps)
    plan.close()
    return {"requests": len(tensors), "elements": total,
            "graph_ms": round(ms_b, 4), "graph_gelem_s": round(total / ms_b / 1e6, 2),
            "per_function_launches_ms": round(ms_s, 4),
            "per_function_gelem_s": round(total / ms_s / 1e6, 2)}


def extra_autograd(lib, L, stream, reps, n=1 << 24):
    """Forward + backward kernels of the autograd functions, binary32,
    U[0.1, 10] operands."""
    import torch
    import workloads as W
    sh = stream.cuda_stream
    res = {}
    for fn in ("sin", "exp", "log", "tanh", "pow", "atan2"):
        a = torch.from_numpy(W.autograd_inputs(fn, n, 0)).cuda()
        b = torch.from_numpy(W.autograd_inputs(fn, n, 1)).cuda()
        g = torch.from_numpy(W.autograd_inputs(fn, n, 2)).cuda()
        y = torch.empty_like(a)
        g0 = torch.empty_like(a)
        g1 = torch.empty_like(a)
        fwd = getattr(lib, L.entry_name(fn, "u10", "f32"))
        bwd = getattr(lib, "libm_hip_%s_u10_f32_bwd" % fn)
        if fn in ("pow", "atan2"):
            cf = checked(lib, fn, fwd, a.data_ptr(), b.data_ptr(), y.data_ptr(), n, sh)
            cb = checked(lib, fn + "_bwd", bwd, a.data_ptr(), b.data_ptr(), g.data_ptr(),
                         g0.data_ptr(), g1.data_ptr(), n, sh)
            nbytes = 4 * 5
        else:
            cf = checked(lib, fn, fwd, a.data_ptr(), y.data_ptr(), n, sh)
            cb = checked(lib, fn + "_bwd", bwd, a.data_ptr(), g.data_ptr(), g0.data_ptr(), n, sh)
            nbytes = 4 * 3
        ms_f, ms_b = time_launches(stream, [cf, cb], reps)
        res[fn] = {"fwd_ms": round(ms_f, 4), "bwd_ms": round(ms_b, 4),
                   "fwd_bwd_gelem_s": round(n / (ms_f + ms_b) / 1e6, 2),
                   "bwd_hbm_frac": round(nbytes * n / (ms_b * 1e-3) / HBM_PEAK, 4)}
    return {"n": n, "dtype": "f32", "functions": res}


def extra_share(lib, L, stream, calls, n_share, reps):
    """The whole step at one GPU's share of an eight-way split: the first
    n_share elements of every array (launch shapes from the table for that
    size, the defaults unless tuned)."""
    shares = []
    for item, f, cargs in calls:
        shares.append(checked(lib, L.entry_name(*item), f, *(cargs[:-2] + (n_share, cargs[-1]))))

    def run_all():
        for g in shares:
            g()
    ms = time_launches(stream, [run_all], reps)[0]
    return {"elements_per_kernel": n_share, "ms_per_step": round(ms, 4),
            "gelem_s": round(n_share * len(calls) / ms / 1e6, 2)}


def extra_inverse_trig(lib, L, stream, n, reps, ops):
    """asin, acos, atan (u10 and u35) and log u35, binary64 and binary32, on
    2^26 elements each: asin/acos on the unit-interval mixture, atan and log
    on the mixture; per kernel the same roofline fractions as the step's."""
    import torch
    import workloads as W
    sh = stream.cuda_stream
    res = {}
    for fn in ("asin", "acos", "atan", "log"):
        for dt in ("f64", "f32"):
            a = W.function_mixture(fn, dt, n, 0)
            ta = torch.from_numpy(a).cuda()
            to = torch.empty_like(ta)
            for v in (("u35",) if fn == "log" else ("u10", "u35")):
                nm = L.entry_name(fn, v, dt)
                ms = time_launches(stream, [checked(lib, nm, getattr(lib, nm), ta.data_ptr(),
                                                    to.data_ptr(), n, sh)], reps)[0]
                vo, v64, _ = valu_ops(fn, v, dt, a, ops)
                slots = max(v64, vo / 2)
                nb = ESIZE[dt] * 2
                res["%s_%s_%s" % (fn, v, dt)] = {
                    "ms": round(ms, 4), "gelem_s": round(n / ms / 1e6, 2),
                    "valu_per_elem": vo, "valu_f64_per_elem": v64,
                    "hbm_frac": round(nb * n / HBM_PEAK / (ms * 1e-3), 4),
                    "alu_frac": round(slots * n / VALU_SLOTS / (ms * 1e-3), 4)}
            del ta, to
    return res


C99_EXTRA = [(fn, "u10") for fn in ("log10", "log1p", "exp10", "expm1", "cbrt", "hypot", "asinh",
                                    "acosh", "atanh", "erf", "erfc")]
U35_EXTRA = [(fn, "u35") for fn in ("atan2", "sinh", "cosh", "tanh")]


def extra_functions(lib, L, stream, n, reps, ops, kinds):
    """Further function-variants, binary64 and binary32, on 2^26 elements of
    each function's mixture (two operands for binary functions); per kernel
    the same roofline fractions as the step's."""
    import torch
    import workloads as W
    sh = stream.cuda_stream
    res = {}
    for fn, var in kinds:
        binary = fn in L.BINARY
        for dt in ("f64", "f32"):
            a = W.function_mixture(fn, dt, n, 0)
            ta = torch.from_numpy(a).cuda()
            to = torch.empty_like(ta)
            nm = L.entry_name(fn, var, dt)
            if binary:
                tb = torch.from_numpy(W.function_mixture(fn, dt, n, 1)).cuda()
                args = (ta.data_ptr(), tb.data_ptr(), to.data_ptr(), n, sh)
            else:
                tb = None
                args = (ta.data_ptr(), to.data_ptr(), n, sh)
            ms = time_launches(stream, [checked(lib, nm, getattr(lib, nm), *args)], reps)[0]
            vo, v64, _ = valu_ops(fn, var, dt, a, ops)
            slots = max(v64, vo / 2)
            nb = ESIZE[dt] * (3 if binary else 2)
            res["%s_%s_%s" % (fn, var, dt)] = {
                "ms": round(ms, 4), "gelem_s": round(n / ms / 1e6, 2),
                "valu_per_elem": vo, "valu_f64_per_elem": v64,
                "hbm_frac": round(nb * n / HBM_PEAK / (ms * 1e-3), 4),
                "alu_frac": round(slots * n / VALU_SLOTS / (ms * 1e-3), 4)}
            del ta, tb, to
    return res


def fmod_valu(L, fn, dt, a, b, ops, m=1 << 20):
    """Dynamic VALU work per element of fmod / remainder: the long-division
    loop runs, for each element slot of a pack, as many digit steps as the
    slowest of the wave's 64 lanes needs.  Step counts come from the host
    build of the same evaluators (libm_hip_host_fmod_steps) on the first m
    elements; a wave covers 64 consecutive packs of 16 bytes.  VALU per
    element = (whole function - one step) + one step x mean wave steps.
    Returns (valu, valu_f64, wave steps per element, lane steps per element)."""
    import numpy as np
    npd = np.float64 if dt == "f64" else np.float32
    x = np.ascontiguousarray(a[:m], dtype=npd)
    y = np.ascontiguousarray(b[:m], dtype=npd)
    if fn == "remainder":
        with np.errstate(over="ignore"):
            y = y + y                                 # remainder runs fmod(|x|, 2|y|)
    _, st = L.host_fmod_steps(x, y)
    ept = 16 // ESIZE[dt]
    wave = st[: (st.size // (64 * ept)) * 64 * ept].reshape(-1, 64, ept).max(axis=1)
    pre = "p64_" if dt == "f64" else "p32_"
    whole, step = ops[pre + fn], ops[pre + "fmodstep"]
    wm = float(wave.mean())
    vo = whole["valu"] - step["valu"] + step["valu"] * wm
    v64 = whole["valu_f64"] - step["valu_f64"] + step["valu_f64"] * wm
    return vo, v64, wm, float(st.mean())


def extra_paper_domains(lib, L, stream, n, reps, ops):
    """The paper's own benchmark domains (Section 7, table of reciprocal
    throughputs), binary64, 2^26 uniform elements each: sin, cos, tan (u10,
    u35) on U[0.4, 0.5], U[0, 6.28], U[0, 1e100]; asin, acos on U[-1, 1];
    atan on U[-700, 700]; log on U[0, 1e300]; exp on U[-700, 700]; pow on
    U[-30, 30]^2."""
    import torch
    import workloads as W
    sh = stream.cuda_stream
    res = {}
    rows = [(fn, v, dom) for fn in ("sin", "cos", "tan") for v in ("u10", "u35")
            for dom in W.PAPER_DOMAINS[fn]]
    rows += [("asin", v, (-1.0, 1.0)) for v in ("u10", "u35")]
    rows += [("acos", v, (-1.0, 1.0)) for v in ("u10", "u35")]
    rows += [("atan", v, (-700.0, 700.0)) for v in ("u10", "u35")]
    rows += [("log", v, dom) for v in ("u10", "u35") for dom in W.PAPER_DOMAINS["log"]]
    rows += [("exp", "u10", dom) for dom in W.PAPER_DOMAINS["exp"]]
    rows += [("pow", "u10", dom) for dom in W.PAPER_DOMAINS["pow"]]
    for fn, v, (lo, hi) in rows:
        ta = torch.from_numpy(W.paper_domain(fn, lo, hi, n, "f64", 0)).cuda()
        to = torch.empty_like(ta)
        nm = L.entry_name(fn, v, "f64")
        if fn in L.BINARY:
            tb = torch.from_numpy(W.paper_domain(fn, lo, hi, n, "f64", 1)).cuda()
            args = (ta.data_ptr(), tb.data_ptr(), to.data_ptr(), n, sh)
        else:
            tb = None
            args = (ta.data_ptr(), to.data_ptr(), n, sh)
        ms = time_launches(stream, [checked(lib, nm, getattr(lib, nm), *args)], reps)[0]
        nb = 8 * (3 if fn in L.BINARY else 2)
        res["%s_%s_f64 [%g, %g]" % (fn, v, lo, hi)] = {
            "ms": round(ms, 4), "gelem_s": round(n / ms / 1e6, 2),
            "hbm_frac": round(nb * n / HBM_PEAK / (ms * 1e-3), 4)}
        del ta, tb, to
    return res


def extra_fmod_ratio_sweep(lib, L, stream, reps, ops, n=1 << 24):
    """The paper's fmod benchmark (Section 7, the fmod figure): binary64
    fmod with d ~ U[1, 100] and n = r d U[0.95, 1.05] for r = 10^0, 10^0.5,
    ..., 10^25, 2^24 elements per point; time, mean wave steps (the loop
    count the slowest lane of each wave sets) and VALU fraction."""
    import numpy as np
    import torch
    import workloads as W
    sh = stream.cuda_stream
    res = {}
    nm = L.entry_name("fmod", "exact", "f64")
    for k in range(51):
        e = k / 2.0
        rng = W.rng_for(11, "fmod", k)
        d = rng.uniform(1.0, 100.0, n)
        x = 10.0 ** e * d * rng.uniform(0.95, 1.05, n)
        ta, tb = torch.from_numpy(x).cuda(), torch.from_numpy(d).cuda()
        to = torch.empty_like(ta)
        ms = time_launches(stream, [checked(lib, nm, getattr(lib, nm), ta.data_ptr(),
                                            tb.data_ptr(), to.data_ptr(), n, sh)], reps)[0]
        vo, v64, wm, em = fmod_valu(L, "fmod", "f64", x, d, ops)
        slots = max(v64, vo / 2)
        res["1e%.1f" % e] = {"ms": round(ms, 4), "gelem_s": round(n / ms / 1e6, 2),
                             "wave_steps_per_elem": round(wm, 3), "valu_per_elem": round(vo, 1),
                             "alu_frac": round(slots * n / VALU_SLOTS / (ms * 1e-3), 4)}
        del ta, tb, to
    return res


def extra_large_args(lib, L, stream, n, reps, ops):
    """The large-argument workload on 2^26 elements: sin, cos, tan (u10,
    u35) on half sign * 10^U[5, log10 max] and half near multiples of pi/2
    (almost every element takes Payne-Hanek), fmod and remainder on operands
    log-uniform over the whole range (long quotient loops); binary64 and
    binary32.  Trig kernels get the step's roofline fractions; fmod and
    remainder get their VALU work from the digit steps their waves take
    (fmod_valu)."""
    import numpy as np
    import torch
    import workloads as W
    sh = stream.cuda_stream
    res = {}
    kinds = [(fn, v) for fn in ("sin", "cos", "tan") for v in ("u10", "u35")]
    kinds += [("fmod", "exact"), ("remainder", "exact")]
    for fn, var in kinds:
        binary = fn in L.BINARY
        for dt in ("f64", "f32"):
            a = W.large_args(fn, dt, n, 0)
            ta = torch.from_numpy(a).cuda()
            to = torch.empty_like(ta)
            nm = L.entry_name(fn, var, dt)
            if binary:
                bh = W.large_args(fn, dt, n, 1)
                tb = torch.from_numpy(bh).cuda()
                args = (ta.data_ptr(), tb.data_ptr(), to.data_ptr(), n, sh)
            else:
                tb = None
                args = (ta.data_ptr(), to.data_ptr(), n, sh)
            ms = time_launches(stream, [checked(lib, nm, getattr(lib, nm), *args)], reps)[0]
            nb = ESIZE[dt] * (3 if binary else 2)
            r = {"ms": round(ms, 4), "gelem_s": round(n / ms / 1e6, 2),
                 "hbm_frac": round(nb * n / HBM_PEAK / (ms * 1e-3), 4)}
            if not binary:
                vo, v64, slow = valu_ops(fn, var, dt, a, ops)
                slots = max(v64, vo / 2)
                r.update({"payne_hanek_share": round(float(slow), 4), "valu_per_elem": vo,
                          "valu_f64_per_elem": v64,
                          "alu_frac": round(slots * n / VALU_SLOTS / (ms * 1e-3), 4)})
            else:
                vo, v64, wsteps, esteps = fmod_valu(L, fn, dt, a, bh, ops)
                slots = max(v64, vo / 2)
                r.update({"valu_per_elem": round(vo, 1), "valu_f64_per_elem": round(v64, 1),
                          "wave_steps_per_elem": round(wsteps, 3),
                          "lane_steps_per_elem": round(esteps, 3),
                          "alu_frac": round(slots * n / VALU_SLOTS / (ms * 1e-3), 4)})
            res["%s_%s_%s" % (fn, var, dt)] = r
            del ta, tb, to
    return res


def extra_sincos(lib, L, stream, n, reps):
    """sincos u10 (one pass, two outputs) against sin u10 and cos u10 launched
    separately, on the same 2^26-element mixture (binary64, binary32)."""
    import torch
    import workloads as W
    sh = stream.cuda_stream
    res = {}
    for dt in ("f64", "f32"):
        ta = torch.from_numpy(W.function_mixture("sin", dt, n, 0)).cuda()
        ts, tc = torch.empty_like(ta), torch.empty_like(ta)
        nm = "libm_hip_sincos_u10_%s" % dt
        one = checked(lib, nm, getattr(lib, nm), ta.data_ptr(), ts.data_ptr(), tc.data_ptr(), n, sh)
        calls = [checked(lib, L.entry_name(fn, "u10", dt), getattr(lib, L.entry_name(fn, "u10", dt)),
                         ta.data_ptr(), out.data_ptr(), n, sh)
                 for fn, out in (("sin", ts), ("cos", tc))]

        def both():
            for g in calls:
                g()
        ms_one, ms_two = time_launches(stream, [one, both], reps)
        res[dt] = {"sincos_ms": round(ms_one, 4), "sin_plus_cos_ms": round(ms_two, 4),
                   "gelem_s": round(n / ms_one / 1e6, 2),
                   "speedup": round(ms_two / ms_one, 3)}
        del ta, ts, tc
    return res


def extra_sorted_paths(lib, L, stream, host, n, reps):
    """Ablation: the trig kernels on the same inputs sorted so that
    Cody-Waite and Payne-Hanek elements never share a wave, against the
    mixed order of the step (the cost of path divergence)."""
    import numpy as np
    import torch
    sh = stream.cuda_stream
    res = {}
    for fn in ("sin", "tan"):
        for dt in ("f64", "f32"):
            a = host[(fn, "u10", dt)][0]
            order = np.argsort(~(np.abs(a) < SLOW_TRIG[dt]), kind="stable")
            ts = torch.from_numpy(np.ascontiguousarray(a[order])).cuda()
            tm = torch.from_numpy(a).cuda()
            to = torch.empty_like(ts)
            nm = L.entry_name(fn, "u10", dt)
            f = getattr(lib, nm)
            ms_m, ms_s = time_launches(stream, [
                checked(lib, nm, f, tm.data_ptr(), to.data_ptr(), n, sh),
                checked(lib, nm, f, ts.data_ptr(), to.data_ptr(), n, sh)], reps)
            res["%s_u10_%s" % (fn, dt)] = {"mixed_ms": round(ms_m, 4), "sorted_ms": round(ms_s, 4),
                                           "speedup_sorted": round(ms_m / ms_s, 3)}
            del ts, tm, to
    return res


def extra_small_set(lib, L, stream, reps, ops):
    """The binary64 small set (2^20 elements: sin, cos, exp on U[-10, 10],
    log on (0, 1000]), 8 MiB per array: resident in the 256 MiB last-level
    cache when timed back to back (warm), so the VALU fraction is the one to
    read."""
    import torch
    import workloads as W
    sh = stream.cuda_stream
    res = {}
    n = 1 << 20
    for fn in ("sin", "cos", "exp", "log"):
        a = W.small_set(fn, n)
        ta = torch.from_numpy(a).cuda()
        to = torch.empty_like(ta)
        nm = L.entry_name(fn, "u10", "f64")
        f = checked(lib, nm, getattr(lib, nm), ta.data_ptr(), to.data_ptr(), n, sh)
        f()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(20 * reps):
            f()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / (20 * reps)
        vo, v64, _ = valu_ops(fn, "u10", "f64", a, ops)
        slots = max(v64, vo / 2)
        res[fn] = {"us": round(ms * 1e3, 2), "gelem_s": round(n / ms / 1e6, 2),
                   "alu_frac": round(slots * n / VALU_SLOTS / (ms * 1e-3), 4)}
    return res


def host_cpu_info():
    """CPU model name and the number of CPUs this process may use."""
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        nproc = os.cpu_count() or 1
    return cpu, nproc


def cpu_baseline(inputs, sample):
    """The oracle as it stands, on the first ``sample`` elements of every
    (function, dtype) input of the step, over a process pool on the host's
    cores; the pool is terminated and joined before returning."""
    import oracle
    from oracle.batch import default_workers, shutdown
    workers = default_workers()
    total = 0
    t0 = time.perf_counter()
    try:
        for (fn, v, dt), (a, b) in inputs.items():
            oracle.evaluate(fn, dt, a[:sample], None if b is None else b[:sample],
                            workers=workers)
            total += min(sample, a.shape[0])
    finally:
        shutdown()
    dt_s = time.perf_counter() - t0
    cpu, nproc = host_cpu_info()
    rate = total / dt_s
    return {"value": round(rate / 1e9, 7), "unit": "Gelem/s", "cores": workers,
            "nproc": nproc, "kind": "oracle", "host_cpu": cpu,
            "per_core_Melem_s": round(rate / workers / 1e6, 4),
            "sample": "first %d elements of each of the %d (function, dtype) inputs of the "
                      "step (%d elements, %.1f s, %d worker processes)"
                      % (sample, len(inputs), total, dt_s, workers)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (every element is independent, so G GPUs "
              "would each take 1/G of every array); run with --gpus 1", file=sys.stderr)
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

    tuned = {}
    if not args.no_tune:
        for item, f, cargs in calls:
            fn, v, dt = item
            ta, tb, to = dev[item]
            blk, pk = L.tune(fn, ta, tb, variant=v, out=to)
            tuned["%s_%s_%s" % item] = [blk, pk]
        torch.cuda.synchronize()

    def step():
        for item, f, cargs in calls:
            st = f(*cargs)
            if st != 0:
                raise RuntimeError("%s: %s" % (item, lib.libm_hip_last_error()))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: one event before every launch and one after the last, all
    # on the launch stream; kernel i of step s lasts ev[s][i] -> ev[s][i + 1]
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(calls) + 1)]
           for _ in range(args.steps)]
    for s_i in range(args.steps):
        row = evs[s_i]
        for i, (item, f, cargs) in enumerate(calls):
            row[i].record(stream)
            st = f(*cargs)
            if st != 0:
                raise RuntimeError("%s: %s" % (item, lib.libm_hip_last_error()))
        row[-1].record(stream)
    torch.cuda.synchronize()
    ms_total = evs[0][0].elapsed_time(evs[-1][-1])
    ms_step = ms_total / args.steps
    elems = n * len(plan)
    value = elems / (ms_step * 1e-3) / 1e9
    print("bench: %.3f ms per step" % ms_step, file=sys.stderr, flush=True)

    with open(OPS_FILE) as fh:
        ops = json.load(fh)
    traffic = load_traffic()
    per = {}
    for i, (item, f, cargs) in enumerate(calls):
        ms = sum(evs[s_i][i].elapsed_time(evs[s_i][i + 1]) for s_i in range(args.steps)) \
            / args.steps
        fn, v, dt = item
        nb = ESIZE[dt] * (3 if fn in BINARY else 2)
        vo, v64, slow = valu_ops(fn, v, dt, host[item][0], ops)
        slots = max(v64, vo / 2)
        t_hbm = nb * n / HBM_PEAK
        t_alu = slots * n / VALU_SLOTS
        rec = {"ms": round(ms, 4), "gelem_s": round(n / ms / 1e6, 2),
               "bytes_per_elem": nb, "valu_per_elem": round(vo, 1),
               "valu_f64_per_elem": round(v64, 1), "valu_slots_per_elem": round(slots, 1),
               "hbm_frac": round(t_hbm / (ms * 1e-3), 4),
               "alu_frac": round(t_alu / (ms * 1e-3), 4),
               "bound": "alu" if t_alu > t_hbm else "hbm"}
        if slow:
            rec["payne_hanek_share"] = round(slow, 4)
        per["%s_%s_%s" % item] = rec
    dom = max(per, key=lambda k: per[k]["ms"])
    fn, v, dt = dom.split("_")
    d = per[dom]
    dom_s = d["ms"] * 1e-3
    tr = traffic.get(dom)
    common = {"kernel": dom, "elements_per_launch": n, "avg_launch_ms": d["ms"],
              "traffic": tr["bytes_per_launch"] if tr else None,
              "traffic_unit": "bytes per launch",
              "algorithmic_bytes_per_launch": d["bytes_per_elem"] * n}
    if d["bound"] == "alu":
        achieved = d["valu_per_elem"] * n / dom_s
        peak = VALU_SLOTS * d["valu_per_elem"] / d["valu_slots_per_elem"]
        roofline = {"bound": "alu", "achieved": round(achieved / 1e12, 2),
                    "peak": round(peak / 1e12, 2), "unit": "T VALU lane-op/s",
                    "frac": round(achieved / peak, 4),
                    "valu_per_elem": d["valu_per_elem"],
                    "valu_f64_per_elem": d["valu_f64_per_elem"], "hbm_frac": d["hbm_frac"]}
    else:
        achieved = d["bytes_per_elem"] * n / dom_s
        roofline = {"bound": "hbm", "achieved": round(achieved / 1e9, 1),
                    "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK, 4), "alu_frac": d["alu_frac"]}
    roofline.update(common)

    # copy ceiling: a plain elementwise copy-like kernel (negation) over the
    # same number of binary64 elements, 16 bytes per element
    src = dev[calls[0][0]][0]
    dst = torch.empty_like(src)
    copy_ms = time_launches(stream, [lambda: torch.neg(src, out=dst)], args.reps)[0]
    copy_gbs = 16 * n / (copy_ms * 1e-3) / 1e9
    del dst

    result = {"metric": "Gelem/s per function at <=1.0/3.5 ULP; % of HBM or VALU roofline",
              "value": round(value, 3), "unit": "Gelem/s", "n_gpus": 1,
              "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "dtype": "f64+f32", "data": "synthetic",
              "config": {"workload": "15 function-variants x {f64, f32} on 2^26 elements "
                                     "each; per element 49% U[-1e4, 1e4], 50% sign*10^U[-300, "
                                     "300] (f32: [-38, 38]), 1% special values",
                         "elements_per_step": elems, "functions": len(plan),
                         "parallelism": "single GPU"},
              "roofline": roofline,
              "copy_ceiling": {"GB_s": round(copy_gbs, 1), "frac_of_peak":
                               round(copy_gbs * 1e9 / HBM_PEAK, 4),
                               "kernel": "torch.neg, f64, 2^26 elements"},
              "per_function": per}
    if tuned:
        result["tuned_launch_shapes"] = tuned
    extras = {}
    if not args.no_extras and not args.only:
        t_x = time.perf_counter()

        def extra(name, f, *fa):
            extras[name] = f(*fa)
            # every extra goes to stderr as it completes (and to the full file)
            print("bench-extra %s %s" % (name, json.dumps(extras[name])), file=sys.stderr,
                  flush=True)
        with open(OPS_FILE) as fh:
            ops = json.load(fh)
        extra("precision_forms", extra_precision_forms, lib, L, stream, dev, n, args.narrow_n,
              args.reps)
        extra("batch", extra_batch, lib, L, stream, args.reps)
        extra("autograd", extra_autograd, lib, L, stream, args.reps)
        extra("per_gpu_share", extra_share, lib, L, stream, calls, n // 8, args.reps)
        extra("inverse_trig", extra_inverse_trig, lib, L, stream, n, args.reps, ops)
        extra("c99_functions", extra_functions, lib, L, stream, n, args.reps, ops, C99_EXTRA)
        extra("u35_forms", extra_functions, lib, L, stream, n, args.reps, ops, U35_EXTRA)
        extra("sincos", extra_sincos, lib, L, stream, n, args.reps)
        extra("large_args", extra_large_args, lib, L, stream, n, args.reps, ops)
        extra("paper_domains", extra_paper_domains, lib, L, stream, n, args.reps, ops)
        extra("fmod_ratio_sweep", extra_fmod_ratio_sweep, lib, L, stream, args.reps, ops)
        extra("trig_sorted_by_path", extra_sorted_paths, lib, L, stream, host, n, args.reps)
        extra("small_set_f64_warm", extra_small_set, lib, L, stream, args.reps, ops)
        print("bench: extras in %.1f s" % (time.perf_counter() - t_x), file=sys.stderr,
              flush=True)
    result.update(extras)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(host, args.cpu_sample)
    if args.out:
        d = os.path.dirname(os.path.abspath(args.out))
        os.makedirs(d, exist_ok=True)
        with open(args.out, "w") as fh:
            json.dump(result, fh, indent=1)
    print(json.dumps(compact(result, args.out)))


def compact(result, full_path):
    """The one stdout line: the contract's keys, the roofline object, the
    CPU baseline and per kernel (Gelem/s, HBM fraction, VALU fraction); the
    extras stay in the full file."""
    keep = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
            "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
            "roofline")
    out = {k: result[k] for k in keep}
    if "cpu_baseline" in result:
        out["cpu_baseline"] = result["cpu_baseline"]
    out["copy_ceiling_frac"] = result["copy_ceiling"]["frac_of_peak"]
    out["per_function"] = {"columns": ["gelem_s", "hbm_frac", "alu_frac"]}
    for k, r in result["per_function"].items():
        out["per_function"][k] = [r["gelem_s"], round(r["hbm_frac"], 3), round(r["alu_frac"], 3)]
    if full_path:
        out["full_results"] = full_path
    return out


if __name__ == "__main__":
    main()
