"""Build the simulator's shared library in-tree for gfx950.

    python -m paper_2605_15098_amd.build

Produces ``paper_2605_15098_amd/libsvmi.so`` from ``csrc/`` with hipcc. The
packed-FP32 target feature is switched off for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsvmi.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.environ.get("HIPCC", os.path.join(ROCM, "bin", "hipcc"))

SOURCES = ["kernels.hip", "api.cpp", "plan.cpp"]
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, src + ".o")
        cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-c", path, "-o", obj,
               "-Wall", "-Wno-unused-function"]
        if src.endswith(".hip"):
            cmd += DEVICE_FLAGS
        else:
            # host-only translation units: plain g++ against the HIP runtime headers
            cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-c", path, "-o", obj, "-Wall",
                   "-Wno-unused-result", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
