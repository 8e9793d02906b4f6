"""Build libclb.so (HIP for gfx950) in-tree: ``python -m paper_1710_10569_amd.build``
(``--poison``: the debug variant libclb_poison.so used by the tests).

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
# debug variant for the tests: populations whose source lies beyond a wall are loaded as NaN
LIB_POISON = os.path.join(HERE, "libclb_poison.so")
SOURCES = ["clb.hip", "clb_batch.hip", "clb3d.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics"]


def build(verbose: bool = False, extra=(), poison: bool = False) -> str:
    """Build libclb.so, or with poison=True the debug variant libclb_poison.so."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    out = LIB_POISON if poison else LIB
    cmd = [HIPCC, *FLAGS, *(["-DCLB_POISON_UNKNOWN"] if poison else []), *extra, "-shared", "-o", out + ".tmp", *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "--poison"]
    build(verbose=True, extra=args, poison="--poison" in sys.argv[1:])
