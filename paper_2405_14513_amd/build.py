"""Build libbk.so (HIP kernels for gfx950 + C ABI + host tables) in-tree.

Usage: python -m paper_2405_14513_amd.build   (or call build()).
The host geometry (bk_tables.cpp) is compiled with g++ and
-ffp-contract=off so its float64 bin decisions are plain IEEE operations; the
device code is compiled with hipcc for gfx950 only, with packed-FP32
instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libbk.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang",
    "-target-feature",
    "-Xclang",
    "-packed-fp32-ops",
]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return res


def build(verbose: bool = False) -> str:
    """Compile every source and link libbk.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    o_tables = os.path.join(BUILD, "bk_tables.o")
    o_api = os.path.join(BUILD, "bk_api.o")
    steps = [
        ["g++", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-c",
         os.path.join(CSRC, "bk_tables.cpp"), "-o", o_tables],
        [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "bk_api.hip"), "-o", o_api],
        [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", o_api, o_tables, "-o", LIB + ".tmp", "-lpthread"],
    ]
    for cmd in steps:
        if verbose:
            print(" ".join(cmd), flush=True)
        _run(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
