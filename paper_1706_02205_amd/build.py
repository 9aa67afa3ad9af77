"""Build libkchol.so (host analysis + gfx950 HIP kernels + C ABI) in-tree.

    python -m paper_1706_02205_amd.build [-v]

The host analysis is plain C++17 (g++); the kernels and the C ABI are compiled
by hipcc for gfx950 only.  Both use -ffp-contract=off so that no multiply and
add are fused unless the source writes an fma.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libkchol.so")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-pthread", "-Wall", "-Wextra",
              "-Wno-unused-parameter"]
# -amdgpu-mfma-vgpr-form: matrix-core accumulators live in ordinary VGPRs, so the
# dense product's accumulators are not copied to and from AGPRs around each MFMA.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-mfma-vgpr-form=1",
             "-Wno-unused-command-line-argument"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", INCLUDE, "-I", CSRC]
    objs = []
    for src in ("analysis.cpp",):
        obj = os.path.join(BUILD, src + ".o")
        _run(["g++", *HOST_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    for src in ("kchol.hip", "pcg.hip"):
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC, *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp, "-pthread"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
