"""Build the CPU oracle library (test infrastructure only).

    python -m oracle.build

gcc, FP64, no contraction of products into fused multiply-adds, OpenMP over
pixel chunks.  The output is oracle/liboracle.so.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "dsgm_oracle.c"), os.path.join(HERE, "preprocess_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c99", "-Wall", "-Wextra", "-o", LIB + ".tmp"] + SRCS + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
