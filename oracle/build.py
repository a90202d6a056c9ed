"""Build the CPU FP64 oracle shared library (test infrastructure only).

The oracle is compiled with ``-O2 -ffp-contract=off -fno-fast-math`` so that
every floating-point expression is evaluated exactly as written (no FMA
contraction, no reassociation).  Run ``python oracle/build.py``; the package's
build entry point calls :func:`build` as well.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["adscl_oracle.c", "adscl_oracle_adj.c"]
LIB = os.path.join(HERE, "liboracle.so")
FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11",
         "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose=False):
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["gcc"] + FLAGS + srcs + ["-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
