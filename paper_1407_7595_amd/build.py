"""Build libmem.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "mem_lib.hip")
LIB = os.path.join(HERE, "libmem.so")
ARCH = os.environ.get("MEM_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for the device code (the compiler
# would otherwise form them from scalar or float2 code).
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=fast", "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def build(verbose=False, extra=()):
    cmd = ["hipcc"] + FLAGS + list(extra) + ["-o", LIB, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
