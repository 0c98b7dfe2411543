"""Count the vector ALU instructions of every evaluator path on gfx950.

Compiles ``op_probe.hip`` (one kernel per path: Cody-Waite reduction,
Payne-Hanek, polynomial + reconstruction, whole functions) to assembly and
counts, per kernel, the VALU instructions, those of them that run on the
binary64 units, the transcendental-unit instructions, and the
floating-point operations (an FMA counts as two).  The result,
``valu_per_element.json``, is the per-element work the benchmark uses for
the ALU roofline of compute-bound kernels: one element per lane, so VALU
instructions per kernel = lane-operations per element.  The probes are
built with LMH_COUNT_COMMON_PATH, which drops the paths only rare arguments
take (results in the subnormal range), so the counts are those of the path
almost every wave runs.  fmod and remainder loop: ``p64_fmodstep`` /
``p32_fmodstep`` count one digit step, and the whole-function probes hold
one copy of it; the benchmark scales by the steps the waves actually take.

Run:  python -m paper_2001_09258_amd.gen.count_ops
"""
import json
import os
import re
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "valu_per_element.json")


def count(asm):
    pat = re.compile(r"^(_Z\S+):\s*;", re.M)
    res = {}
    for m in pat.finditer(asm):
        name = re.sub(r"^_Z\d+", "", m.group(1))
        name = re.sub(r"PK[df]P[df]$", "", name)
        end = asm.find(".Lfunc_end", m.start())
        ins = []
        for line in asm[m.start():end].split("\n")[1:]:
            t = line.strip()
            if not t or t.startswith((".", ";", "//")) or t.endswith(":"):
                continue
            ins.append(t.split()[0])
        prec = "f64" if name.startswith("p64") else "f32"

        def c(rx):
            return sum(1 for x in ins if re.fullmatch(rx, x))
        fma = c(r"v_(fma|fmac|fmaak|fmamk)_%s(_e32|_e64)?" % prec)
        mul = c(r"v_mul_%s(_e32|_e64)?" % prec)
        add = c(r"v_(add|sub|subrev)_%s(_e32|_e64)?" % prec)
        # the probe's own load/store and index arithmetic is a handful of
        # VALU instructions; they are part of every real kernel too
        valu = [x for x in ins if x.startswith("v_")]
        res[name] = {"valu": len(valu),
                     # instructions of the binary64 units (arithmetic, compare,
                     # convert, ldexp/frexp, rounding): at most 64 lanes per
                     # clock per CU, whereas other VALU instructions can
                     # dual-issue
                     "valu_f64": sum(1 for x in valu if "f64" in x),
                     "trans": sum(1 for x in valu if re.match(
                         r"v_(rcp|rsq|sqrt|exp|log|sin|cos)_", x)),
                     "flops": 2 * fma + mul + add}
    return res


def main():
    src = os.path.join(HERE, "op_probe.hip")
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "probe.s")
        subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17",
                        "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
                        "-DLMH_COUNT_COMMON_PATH", "-Xclang",
                        "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only",
                        "-S", "-o", out, src], check=True)
        res = count(open(out).read())
    with open(OUT, "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)
    for k, v in sorted(res.items()):
        print("%-14s valu %4d f64 %4d trans %2d flops %4d"
              % (k, v["valu"], v["valu_f64"], v["trans"], v["flops"]))


if __name__ == "__main__":
    main()
