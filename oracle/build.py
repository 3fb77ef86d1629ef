"""Build the CPU oracle library (test infrastructure only).

gcc, FP64, -O2, OpenMP, no fast-math and no FMA contraction, so the oracle
evaluates its formulas in the order they are written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "numa_oracle.c")
LIB = os.path.join(HERE, "libnuma_oracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
