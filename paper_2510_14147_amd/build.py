"""Compile the HIP library ``libfnn.so`` (in-tree) for gfx950 with hipcc.

All kernels are hand-written HIP for CDNA4; the C ABI is ``include/fnn.h``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfnn.so")
SOURCES = ["runtime.hip", "build.hip", "query.hip", "gram.hip", "learn.hip", "tune.hip",
           "landmark.hip", "api.hip"]

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unused-variable",
         "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False, jobs: int = 4) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs, procs = [], []
    for s in SOURCES:
        o = os.path.join(bdir, s.replace(".hip", ".o"))
        objs.append(o)
        cmd = ["hipcc", "-c", *FLAGS, os.path.join(SRC, s), "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        if len(procs) >= jobs:
            if procs.pop(0).wait():
                raise RuntimeError("hipcc failed")
    for p in procs:
        if p.wait():
            raise RuntimeError("hipcc failed")
    tmp = OUT + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
