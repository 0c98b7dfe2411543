"""Build libm_hip.so (the HIP kernels and the C-ABI) for gfx950 in-tree.

    python -m paper_2001_09258_amd.build

Flags that matter for correctness: -ffp-contract=off (the evaluators place
every FMA explicitly; the paper notes that contraction changes results,
Section 3.3), IEEE denormals kept in binary32 and binary64
(-fno-gpu-flush-denormals-to-zero), no fast-math.  Packed-FP32 instruction
selection is disabled (-packed-fp32-ops).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "batch.hip")]
OUT = os.path.join(HERE, "libm_hip.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero", "-fno-fast-math",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-function"]


def build(verbose=True, extra=()):
    cmd = [HIPCC] + FLAGS + list(extra) + ["-o", OUT + ".tmp"] + SRCS
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(extra=sys.argv[1:])
