"""Compile the CPU oracle into ``oracle/liboracle.so`` with gcc.

FP64 throughout, ``-ffp-contract=off`` so no multiply-add is fused and every
sum keeps its written order; OpenMP only across rows and queries.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "fnn_oracle.c")
    out = os.path.join(HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
           "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-Wall",
           "-Wextra", "-Wno-unused-parameter", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
