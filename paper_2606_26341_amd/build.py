"""Build libhipipm.so for gfx950 with hipcc (in-tree, next to this file).

Each source is compiled to an object of its own in parallel (kernels are launched only from the
source that defines them), then the objects are linked into the shared library."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhipipm.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in
           ("iter_fp64.hip", "iter_mixed.hip", "run_fp64.hip", "run_mixed.hip", "kernels.hip", "api.hip",
            "mlp.hip")]
BUILD_DIR = os.path.join(HERE, "_build")
# the asynchronous-slot kernel loops over whole passes: constants hoisted out of that loop would
# stay live across all of it and spill, so machine-level loop-invariant code motion is off there
# The FP32 + refinement pass kernel holds more small per-lane arrays than the backend's default
# budget for keeping such arrays in registers; past the budget they would live in scratch memory.
EXTRA = {"run_fp64.hip": ["-mllvm", "-disable-machine-licm"],
         "run_mixed.hip": ["-mllvm", "-disable-machine-licm"],
         "iter_mixed.hip": ["-mllvm", "-amdgpu-promote-alloca-to-vector-limit=2048"]}


def hipcc() -> str:
    for p in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in p or os.path.exists(p):
            return p
    return "hipcc"


FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions stay off on this target
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # multiply-adds are fused only where one source expression holds both operations, so
         # that an instance's rounding does not depend on the kernel its code is inlined into
         # (the per-phase, fused and asynchronous-slot kernels give bit-identical iterates)
         "-ffp-contract=on"]


def build_library(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = [os.path.join(BUILD_DIR, os.path.basename(s) + ".o") for s in SOURCES]

    def compile_one(pair):
        src, obj = pair
        cmd = ([hipcc()] + FLAGS + EXTRA.get(os.path.basename(src), [])
               + ["-I", os.path.join(ROOT, "include"), "-c", "-o", obj, src])
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    with ThreadPoolExecutor(len(SOURCES)) as ex:
        list(ex.map(compile_one, zip(SOURCES, objs)))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
    sys.exit(0)
