"""Build the HIP library liblbmhd.so in-tree for gfx950 with hipcc.

hipcc cross-compiles without a GPU, so this runs anywhere ROCm is installed.
Usage: ``python -m paper_1705_09807_amd.build`` or ``build()``.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "liblbmhd.so")

SOURCES = ["lbmhd_kernels.hip", "lbmhd_learned.hip", "lbmhd_api.cpp"]

# Packed FP32 instructions are disabled for all device code; the host pass
# warns that it does not know the feature, which is harmless.
FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    path = os.environ.get("HIPCC") or shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; a ROCm installation is required to build liblbmhd.so")
    return path


def build(verbose: bool = False) -> str:
    """Compile csrc/ into liblbmhd.so (always recompiles).  Returns its path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, "-I", INCLUDE, "-I", CSRC, "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building liblbmhd.so")
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
