"""Compile the plain C oracle into ``oracle/liblbvh_oracle.so`` with gcc.

IEEE binary32 semantics are kept: no contraction into fused multiply-adds,
no fast-math, SSE arithmetic (no x87 excess precision).  OpenMP is on for
the oracle's independent loops (``orc_threads`` picks the thread count; the
default is one).
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbvh_oracle.c")
LIB = os.path.join(HERE, "liblbvh_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-mfpmath=sse", "-msse2", "-fopenmp", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
