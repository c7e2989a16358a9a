"""Build libpitdyn.so in-tree with hipcc for gfx950.

    python paper_1902_00387_amd/build.py

Compiles every HIP source of the library (kernels and C-ABI runtime) into
``paper_1902_00387_amd/libpitdyn.so``.  Always recompiles.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpitdyn.so")
ARCH = os.environ.get("PITDYN_ARCH", "gfx950")

SOURCES = ["kernels.hip", "nn.hip", "pitdyn.cpp", "batch.cpp", "lg.cpp", "io.cpp", "pipeline.cpp", "seed.cpp",
           "static_ws.hip"]

# Packed FP32 instructions are disabled for every HIP translation unit.
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor

    cc = hipcc()
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = [os.path.join(bdir, os.path.splitext(src)[0] + ".o") for src in SOURCES]

    def compile_one(i):
        cmd = [cc, *HIP_FLAGS, "-c", os.path.join(CSRC, SOURCES[i]), "-o", objs[i]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    # translation units compile independently; at most 4 at a time
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as pool:
        list(pool.map(compile_one, range(len(SOURCES))))
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
