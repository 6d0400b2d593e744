"""Compile the CPU oracle (test infrastructure) into oracle/liborc.so.

Plain gcc, FP64, OpenMP.  No GPU code and nothing shared with the HIP
library.  `python oracle/build.py` or `oracle.build.build()`.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orc.c")
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    # -ffp-contract=off: every FP64 operation rounds exactly as written.
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
