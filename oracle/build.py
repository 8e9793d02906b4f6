"""Compile the FP64 CPU oracles (test infrastructure): the two-dimensional one into
``oracle/libclb_oracle.so`` and the three-dimensional one into ``oracle/libclb3d_oracle.so``.

Plain C11 with gcc -O2 and OpenMP over lattice rows; no intrinsics, no fast-math.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "clb_oracle.c")
LIB = os.path.join(HERE, "libclb_oracle.so")
SRC3 = os.path.join(HERE, "clb3d_oracle.c")
LIB3 = os.path.join(HERE, "libclb3d_oracle.so")


def build(verbose: bool = False) -> str:
    for src, lib in ((SRC, LIB), (SRC3, LIB3)):
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-o", lib + ".tmp", src, "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(lib + ".tmp", lib)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
