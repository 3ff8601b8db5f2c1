"""Build libkfmi.so (HIP, gfx950) in-tree with hipcc.

Run as `python -m paper_2105_01796_amd.build` or call build().  The library
is compiled every time build() is called.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libkfmi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# the fit kernels of each field kind and stepping precision compile in a
# translation unit of their own, all in parallel
FIT_UNITS = [f"kf_fit_{fk}_{p}.hip" for fk in ("uniform", "solenoid", "map") for p in ("fp64", "mixed")]
SOURCES = [os.path.join(CSRC, f) for f in ["kf_fit.hip", "kf_vjp.hip", *FIT_UNITS]]
OBJDIR = os.path.join(ROOT, "_build")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wno-unused-result",
]


def build(verbose: bool = False, extra=()) -> str:
    """Compile every translation unit (in parallel), then link the library."""
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = os.path.join(OBJDIR, os.path.splitext(os.path.basename(src))[0] + ".o")
        cmd = [HIPCC, *FLAGS, *extra, *inc, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
