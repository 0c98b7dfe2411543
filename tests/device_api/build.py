"""Build the device-API check library (test helper) for gfx950 in-tree.

    python -m tests.device_api.build

Deliberately compiled WITHOUT -ffp-contract=off: the evaluator headers must
keep their own contraction control under the compiler's default mode, as a
user's kernel including include/libm_hip_device.h would be built.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "check.hip")
OUT = os.path.join(HERE, "libdevice_api_check.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose=True):
    cmd = [HIPCC] + FLAGS + ["-o", OUT + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build()
