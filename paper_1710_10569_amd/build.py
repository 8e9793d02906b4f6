"""Build libclb.so (HIP for gfx950) in-tree: ``python -m paper_1710_10569_amd.build``.

Every HIP source is compiled with packed FP32 instructions disabled (-packed-fp32-ops) and linked
into one shared library next to this file.  -ffp-contract=on: a multiply-add is fused only within
one source expression, so every kernel that inlines the same per-node code (any tile shape, the
batch schedules) computes bitwise the same results.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libclb.so")
SOURCES = ["clb.hip", "clb_batch.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics"]


def build(verbose: bool = False, extra=()) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [HIPCC, *FLAGS, *extra, "-shared", "-o", LIB + ".tmp", *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
