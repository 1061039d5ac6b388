"""Build the CPU oracle shared library (test infrastructure only).

gcc, -O2 without fast-math (IEEE semantics are part of the oracle's
contract), OpenMP for the direct sums, libquadmath for the closed forms.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mhk_oracle.c")
LIB = os.path.join(HERE, "liboracle_mhk.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=gnu11", "-Wall",
           "-Wno-unused-function", SRC, "-o", LIB + ".tmp", "-lquadmath", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
