"""Build the oracle's C library (plain gcc, portable x86-64 code).

ORACLE -- test infrastructure.  Kept portable (no -march=native) because the
library is built on one host and may run on another.  OpenMP splits the
oracle's node loops over threads for the CPU baseline's all-core timing; the
results do not depend on the thread count.
"""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mg_ref.c")
LIB = os.path.join(HERE, "libmhs_oracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
