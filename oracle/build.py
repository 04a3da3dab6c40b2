"""Compile the oracle's C sources into oracle/liboracle.so (gcc, OpenMP).

Test infrastructure only.  Strict IEEE single/double arithmetic: no
-ffast-math, no floating-point contraction (the FP32 skeleton must perform
exactly one rounding per written operation).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["keyspec.c", "composite.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
           "-o", LIB] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
