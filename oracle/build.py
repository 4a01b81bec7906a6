"""Build the CPU oracle shared library (plain C, gcc, OpenMP).

-ffp-contract=off keeps every multiply-add separate unless the source asks for
fma() explicitly; -mfma lets those explicit calls use the hardware instruction
(correctly rounded either way).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    out = os.path.join(HERE, "liboracle.so")
    cmd = [
        "gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
        "-mfma", "-fno-math-errno", "-Wall", "-Wextra", "-Wno-unused-parameter",
        os.path.join(HERE, "spdba_oracle.c"), "-o", out + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
