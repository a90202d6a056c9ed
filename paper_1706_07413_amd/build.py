"""Build libadscl.so (HIP, gfx950) in-tree.

Compiles every source under csrc/ with hipcc for gfx950 and links them into
paper_1706_07413_amd/libadscl.so.  Packed FP32 instructions are disabled for
all device code.  Usage: ``python -m paper_1706_07413_amd.build`` (or the
repository's ``__graft_entry__.build()``).
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libadscl.so")
ARCH = os.environ.get("ADSCL_OFFLOAD_ARCH", "gfx950")
SOURCES = ["evolve.hip", "evolve_big.hip", "adjoint.hip", "aux.hip", "spectrum.hip", "noalloc.hip", "scheme.hip", "api.cpp"]
# The forward kernel is latency-bound (one workgroup of two wavefronts per SIMD
# on a CU at P = 8): the machine scheduler's maximum-ILP strategy shortens its
# dependent chains without spilling (1-2% on a step, same arithmetic).
EXTRA = {"evolve.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
         "scheme.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]}


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), "--offload-arch=" + ARCH]
    if src.endswith(".hip"):
        cmd += ["-x", "hip"]
    cmd += common_flags() + EXTRA.get(src, [])
    cmd += ["-I", os.path.join(HERE, "..", "include"), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
