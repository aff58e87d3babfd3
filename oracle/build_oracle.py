"""Builds the FP64 CPU oracle library (test infrastructure only).

The oracle is plain C compiled with gcc, without fast-math and without FMA
contraction, so that its arithmetic is IEEE double in the order written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dsm_oracle.c")
LIB = os.path.join(HERE, "libdsm_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
        "-o", LIB, SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
