"""Build the oracle's C library (test infrastructure; never part of the GPU
library).  ``python -m oracle.build`` or ``build()`` from Python."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ejoin_oracle.c")
LIB = os.path.join(HERE, "libejoin_oracle.so")

# IEEE double arithmetic as written: no contraction into FMA, no fast-math.
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations",
          "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-std=c11"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
