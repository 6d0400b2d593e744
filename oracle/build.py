"""Compile the CPU oracle (test infrastructure) into oracle/liborc.so.

Plain gcc, FP64, OpenMP.  No GPU code and nothing shared with the HIP
library.  `python oracle/build.py` or `oracle.build.build()`.

`python oracle/build.py --sanitize` (or build(sanitize=True)) compiles the
same source with AddressSanitizer and UndefinedBehaviorSanitizer into
oracle/liborc_san.so, which the oracle's wrapper loads instead when
DPD_ORACLE_SANITIZED=1.  Python itself is not instrumented, so the ASan
runtime has to be loaded first:

    LD_PRELOAD=$(gcc -print-file-name=libasan.so) ASAN_OPTIONS=detect_leaks=0 \\
    DPD_ORACLE_SANITIZED=1 python -m pytest tests -m "not gpu"
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "orc.c")
LIB = os.path.join(HERE, "liborc.so")
LIB_SAN = os.path.join(HERE, "liborc_san.so")
# every undefined-behaviour report aborts instead of printing and going on
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    # -ffp-contract=off: every FP64 operation rounds exactly as written.
    out = LIB_SAN if sanitize else LIB
    opt = ["-O1", *SAN_FLAGS] if sanitize else ["-O2"]
    cmd = ["gcc", *opt, "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)
