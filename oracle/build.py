"""Build the CPU FP64 oracle shared libraries (test infrastructure only).

liboracle.so, the parity build, is compiled with ``-O2 -ffp-contract=off
-fno-fast-math`` so that every floating-point expression is evaluated exactly
as written (no FMA contraction, no reassociation).  The timing build of the CPU
baseline (:func:`build_timing`) is the same sources at ``-O3 -march=native``
(still no contraction and no fast-math, so it computes the same numbers); it is
compiled on the machine that runs it, since ``-march=native`` code need not run
on another host.  Both link OpenMP, which only the batch drivers use (one
instance per thread).  Run ``python oracle/build.py``; the package's build
entry point calls :func:`build` as well.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["adscl_oracle.c", "adscl_oracle_adj.c", "adscl_oracle_batch.c", "adscl_oracle_scheme.c"]
LIB = os.path.join(HERE, "liboracle.so")
COMMON = ["-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]
PARITY_FLAGS = ["-O2"] + COMMON
TIMING_FLAGS = ["-O3", "-march=native"] + COMMON
# the self-sensitivity build: the same sources with multiply-adds contracted
# into FMAs wherever the compiler likes (the host's FMA instructions enabled)
CONTRACT_FLAGS = ["-O2", "-march=native", "-ffp-contract=fast"] + [f for f in COMMON if f != "-ffp-contract=off"]


def _gcc(flags, out, verbose):
    cmd = ["gcc"] + flags + [os.path.join(HERE, s) for s in SOURCES] + ["-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def build(verbose=False):
    """The parity build, in-tree."""
    return _gcc(PARITY_FLAGS, LIB, verbose)


def build_timing(out, verbose=False):
    """The -O3 -march=native timing build, written to `out` (a path outside the
    tree, made on the host that will run it)."""
    return _gcc(TIMING_FLAGS, out, verbose)


def build_contract(out, verbose=False):
    """The sources with FMA contraction on (CONTRACT_FLAGS), written to `out`:
    how far two roundings of the same arithmetic drift apart bounds how long a
    parity window can be at a given tolerance."""
    return _gcc(CONTRACT_FLAGS, out, verbose)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
