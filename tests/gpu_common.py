"""Shared helpers of the GPU parity tests: run one entry point on the device
through the binding, run the oracle on the same inputs, compare."""
import numpy as np

import workloads as W
from tests.ulp import compare, exact_compare

BOUND = {"u10": 1.0, "u35": 3.5}
ORACLE_FMT = {"f64": "f64", "f32": "f32", "bf16": "bf16", "f16": "f16",
              "f32_via_f64": "f32"}


def torch_dtype(dt):
    import torch
    return {"f64": torch.float64, "f32": torch.float32, "f32_via_f64": torch.float32,
            "bf16": torch.bfloat16, "f16": torch.float16}[dt]


def to_device(a, dt):
    """numpy values of the format -> device tensor of that format."""
    import torch
    if dt == "bf16":
        t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a).astype(
            {"f64": np.float64, "f32": np.float32, "f32_via_f64": np.float32,
             "f16": np.float16}[dt]))
    return t.cuda()


def to_host(t):
    import torch
    if t.dtype in (torch.bfloat16, torch.float16):
        t = t.float()
    return t.cpu().numpy().astype(np.float64)


def run_gpu(fn, variant, dt, a, b=None):
    import torch
    import paper_2001_09258_amd as L
    ta = to_device(a, dt)
    tb = to_device(b, dt) if b is not None else None
    out = L.evaluate(fn, ta, tb, variant=variant, via_f64=(dt == "f32_via_f64"))
    torch.cuda.synchronize()
    return to_host(out)


def run_oracle(fn, dt, a, b=None):
    import oracle
    return oracle.evaluate(fn, ORACLE_FMT[dt], np.asarray(a, dtype=np.float64),
                           None if b is None else np.asarray(b, dtype=np.float64))


def check(fn, variant, dt, a, b=None, label=""):
    """Runs the entry point on the GPU and compares it with the oracle."""
    return check_values(fn, variant, dt, a, b, run_gpu(fn, variant, dt, a, b), label)


def check_values(fn, variant, dt, a, b, y, label=""):
    """Compares results y (host float64) of fn on (a, b) with the oracle:
    bit-exact for exact functions, else the variant's ULP bound with the
    special classes bit-exact."""
    y = np.asarray(y, dtype=np.float64)
    rn, hi, lo = run_oracle(fn, dt, a, b)
    if variant == "exact":
        bad, idx = exact_compare(y, rn)
        assert bad == 0, "%s %s %s %s: %d mismatches, e.g. x=%r y=%r want %r" % (
            label, fn, variant, dt, bad, a[idx[:3]], y[idx[:3]], rn[idx[:3]])
        return {"n": len(y), "max_ulp": 0.0, "mean_ulp": 0.0}
    bound = BOUND[variant]
    # binary64/binary32 subnormal results are bit-exact; bf16, f16 and the
    # binary32-through-binary64 form round a rounded value once more, so
    # their subnormal mismatches are reported (and held to the bound)
    mode = "exact" if dt in ("f64", "f32") else "report"
    res = compare(y, rn, hi, lo, ORACLE_FMT[dt], bound, subnormal=mode)
    if mode == "report" and res["subnormal_mismatch"]:
        print("%s %s %s %s: %d of %d subnormal results not correctly rounded" % (
            label, fn, variant, dt, res["subnormal_mismatch"], res["subnormal_results"]),
            flush=True)
    if res["violations"] or res["special_mismatch"]:
        idx = res["bad_idx"][:4]
        msg = "%s %s %s %s: max %.3f ulp, %d over %.1f, %d special mismatches; " \
              "x=%r %s y=%r want %r" % (
                  label, fn, variant, dt, res["max_ulp"], res["violations"], bound,
                  res["special_mismatch"], [float(v) for v in np.asarray(a)[idx]],
                  "" if b is None else "b=%r" % [float(v) for v in np.asarray(b)[idx]],
                  [float(v) for v in y[idx]], [float(v) for v in rn[idx]])
        raise AssertionError(msg)
    return res
