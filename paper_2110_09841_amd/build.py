"""Build the HIP library libcvp.so for gfx950 (in-tree).

hipcc compiles the kernels and the C-ABI host code; packed FP32 instructions
are disabled for every device compile.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libcvp.so")

SOURCES = ["cvp_kernels.hip", "cvp_siddon.hip", "cvp_blas.hip", "cvp_nn.hip", "cvp_synth.hip", "cvp_capi.cpp"]
ARCH = os.environ.get("CVP_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + INCLUDE, "-I" + CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        cmd = ["hipcc", "-c", path, "-o", obj] + COMMON + DEVICE
        if src.endswith(".hip"):
            cmd = ["hipcc", "-x", "hip", "-c", path, "-o", obj] + COMMON + DEVICE
        _run(cmd, verbose)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run(["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
