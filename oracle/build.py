"""Compile the oracle's C source into oracle/libtbkpm_oracle.so with gcc.

The oracle is test infrastructure: plain serial C, FP64, no fused multiply-add
contraction, so that its rounding is the textbook one.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tbkpm_oracle.c")
LIB = os.path.join(HERE, "libtbkpm_oracle.so")


def build(verbose=False):
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
