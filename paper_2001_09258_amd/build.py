"""Build libm_hip.so (the HIP kernels and the C-ABI) for gfx950 in-tree, and
libm_hip_host.so (the host build of the bit-consistent evaluators).

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
SRCS = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "batch.hip", "consistent.hip")]
OUT = os.path.join(HERE, "libm_hip.so")
OBJDIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", "g++")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero", "-fno-fast-math",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-function"]

# the host build of the bit-consistent evaluators: no contraction, no
# reassociation, IEEE binary64/binary32 arithmetic (SSE2 on x86-64)
HOST_SRC = os.path.join(HERE, "csrc", "host_scalar.cpp")
HOST_OUT = os.path.join(HERE, "libm_hip_host.so")
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
              "-Wno-unknown-pragmas"]


def build(verbose=True, extra=()):
    """Compile every source to an object (in parallel), then link."""
    os.makedirs(OBJDIR, exist_ok=True)
    procs = []
    objs = []
    for src in SRCS:
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        cmd = [HIPCC] + FLAGS + list(extra) + ["-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    failed = [src for p, src in procs if p.wait() != 0]
    if failed:
        raise RuntimeError("compilation failed: %s" % ", ".join(failed))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", OUT + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    build_host(verbose)
    return OUT


def build_host(verbose=True):
    cmd = [CXX] + HOST_FLAGS + ["-o", HOST_OUT + ".tmp", HOST_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(HOST_OUT + ".tmp", HOST_OUT)
    return HOST_OUT


if __name__ == "__main__":
    build(extra=sys.argv[1:])
