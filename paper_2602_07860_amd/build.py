"""Builds the HIP library (gfx950) in-tree: paper_2602_07860_amd/lib/libmotionblur.so.

hipcc compiles the kernels and the C-ABI host code for gfx950 only.  Packed
FP32 instruction selection is switched off for all device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libmotionblur.so")
SOURCES = [os.path.join(CSRC, "rb_kernels.hip"), os.path.join(CSRC, "rb_api.cpp")]
ARCH = os.environ.get("RB_OFFLOAD_ARCH", "gfx950")


def hipcc_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False, extra=None) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(LIBDIR, os.path.basename(src) + ".o")
        cmd = ["hipcc", "-x", "hip", "-c", src, "-o", obj] + hipcc_flags() + list(extra or [])
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
