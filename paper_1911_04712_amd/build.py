"""Compile the HIP library (gfx950) into paper_1911_04712_amd/libdpd.so.

    python -m paper_1911_04712_amd.build      (or build.build())

The library is plain HIP C++ with a C ABI (include/dpd.h); it links against
nothing but the HIP runtime.  Flags:
  -ffp-contract=off      pair arithmetic uses explicit fmaf only, so every
                         kernel evaluates a pair with the same instructions;
  -packed-fp32-ops off   no v_pk_* FP32 instructions are generated.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libdpd.so")
SOURCES = ["dpd_kernels.hip", "dpd_force.hip", "dpd_capi.hip", "dpd_server.cpp"]
ARCH = os.environ.get("DPD_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


# Sources whose revision keys the autotuner cache: a tile tuned for one
# version of the force kernel is not reused for another.
REV_SOURCES = ["dpd_force.hip", "dpd_device.hpp", "dpd_internal.hpp"]


def kernel_rev() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in REV_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def build(verbose: bool = False, extra=()) -> str:
    objs = []
    rev = kernel_rev()
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), "-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-ffp-contract=off",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC, f'-DDPD_KERNEL_REV="{rev}"', *extra,
               "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        noise = "is not a recognized feature for this target"
        msg = "\n".join(ln for ln in (r.stdout + r.stderr).splitlines() if noise not in ln)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
        if verbose and msg.strip():
            print(msg)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
