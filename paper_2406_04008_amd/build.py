"""Builds libcollage.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libcollage.so")
SOURCES = [os.path.join(PKG, "csrc", "collage_kernels.hip"), os.path.join(PKG, "csrc", "collage_api.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # keep every float operation as written: the scan and the re-decision of the nearest edge must
    # round identically, and every sum runs in a fixed order
    "-ffp-contract=off",
    # no packed FP32 instructions (they are not used by this code and are excluded on purpose)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def build(verbose: bool = False, extra=None) -> str:
    cmd = [HIPCC] + FLAGS + (extra or []) + ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
                                               "-o", LIB + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
