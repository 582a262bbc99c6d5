"""Build the gfx950 library ``liblbmhd.so`` in-tree with hipcc.

Usage: ``python -m paper_1607_08675_amd.build`` (or ``build()`` from Python).
Every HIP source is compiled for gfx950 only, with packed FP32 instructions
disabled (the compiler otherwise forms v_pk_* FP32 ops from scalar code).
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liblbmhd.so")
SOURCES = ["lbmhd_kernels.hip", "lbmhd_adjoint.hip", "lbmhd_capi.hip", "lbmhd3.hip"]
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Wall", "-Wno-unused-command-line-argument",
]


def build(extra_flags=(), out: str = LIB, verbose: bool = False) -> str:
    """Compile every source to an object, then link the shared library."""
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [HIPCC, *COMMON_FLAGS, *extra_flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    for obj in objs:
        os.remove(obj)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
