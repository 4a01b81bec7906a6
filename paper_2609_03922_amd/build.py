"""Build the HIP library libspdba.so for gfx950 (in-tree).

Every HIP translation unit is compiled with -ffp-contract=off (the update core
fixes its own rounding with explicit fma) and with packed FP32 instructions
disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libspdba.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SOURCES = ["spdba_kernels.hip", "spdba_api.cpp", "spdba_proposer.hip", "spdba_rcd.hip", "spdba_mdbp.hip",
           "spdba_static.hip"]
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    objs = []
    os.makedirs(os.path.join(ROOT, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(ROOT, "_build", src + ".o")
        cmd = [os.path.join(ROCM, "bin", "hipcc"), *HIP_FLAGS, "-I", os.path.join(ROOT, "include"),
               "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd.insert(1, "-x")
            cmd.insert(2, "hip")
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    cmd = [os.path.join(ROCM, "bin", "hipcc"), "--offload-arch=gfx950", "-shared", "-fPIC", *objs,
           "-L", os.path.join(ROCM, "lib"), "-lrocfft", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}",
           "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
