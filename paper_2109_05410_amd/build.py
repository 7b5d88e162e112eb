"""Build liboocs.so (HIP for gfx950) in-tree with hipcc.

Every HIP translation unit is compiled without floating-point contraction
(the stencils keep a fixed FP32 operation order), with FP32 denormals
preserved (the codec scales tiny values exactly), and with packed FP32
instructions switched off.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "liboocs.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-I", INC, "-I", CSRC,
]
DEVICE = [
    f"--offload-arch={ARCH}", "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
SOURCES = {
    "kernels.hip": True,   # device code
    "noalloc.hip": True,   # device code (the library-held scratch array) and its entry point
    "codec64.hip": True,   # device code: the FP64 format and the FP64 wave step
    "plan.cpp": False,     # host only
    "host.cpp": False,     # host only (HIP runtime API)
    "adjoint.cpp": False,  # host only (HIP runtime API)
    "batch.cpp": False,    # host only (HIP runtime API)
    "sdma.cpp": False,     # host only (HSA runtime, looked up in-process)
}


def _compile(src: str, device: bool, verbose: bool) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC, "-c"] + COMMON
    if device:
        cmd += DEVICE
    else:
        cmd += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]
    cmd += [os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda kv: _compile(kv[0], kv[1], verbose), SOURCES.items()))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
