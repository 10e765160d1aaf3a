"""Build the oracle shared library (plain C, FP64, no contraction).

Test infrastructure only: the oracle is loaded by the tests, the smoke check
and the CPU-baseline leg of the benchmark, never by the product path.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["philox_vegas.c", "dirac.c", "integrands.c", "driver.c", "flow.c", "phasespace.c", "pdfgrid.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
           "-o", LIB] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
