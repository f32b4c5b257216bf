"""Build the CPU oracle library (liboracle.so) with gcc.

Test infrastructure: the oracle is compiled here so that the test suite, the
smoke check and the CPU-baseline timing can load it.  Flags: -O2 for a
reasonable speed, -ffp-contract=off so that no multiply-add is fused and every
expression rounds as written, -fopenmp for the optional row-parallel sweep.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["mco.c"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-fopenmp", "-Wall", "-Wextra", "-Wno-unused-parameter", "-shared",
           "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
