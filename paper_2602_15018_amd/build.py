"""Build the HIP libraries in-tree with hipcc for gfx950: libnsim_ev.so (the
event path), libnsim_up.so (the learned temporal upsampler) and
libnsim_repr.so (time surface and polarity event frames)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libnsim_ev.so")
SOURCES = ["ev_kernels.hip", "ev_runtime.cpp"]
UP_LIB = os.path.join(PKG, "libnsim_up.so")
UP_SOURCES = ["up_kernels.hip", "up_runtime.cpp"]
REPR_LIB = os.path.join(PKG, "libnsim_repr.so")
REPR_SOURCES = ["repr_kernels.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build_one(lib, sources, verbose=False, extra=()) -> str:
    objs = []
    for src in sources:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-I", CSRC,
               "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs,
           "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


def build(verbose: bool = False, extra=()) -> str:
    """Compile every source and link the libraries (always rebuilds)."""
    build_one(UP_LIB, UP_SOURCES, verbose, extra)
    build_one(REPR_LIB, REPR_SOURCES, verbose, extra)
    return build_one(LIB, SOURCES, verbose, extra)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
