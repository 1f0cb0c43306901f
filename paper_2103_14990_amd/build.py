"""Builds libdlmpc.so in-tree for gfx950 with hipcc (``python -m paper_2103_14990_amd.build``)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libdlmpc.so")
SOURCES = ["setup_host.cpp", "setup_kernels.hip", "admm_kernels.hip", "batch_kernels.hip", "warmstart_kernels.hip", "dlmpc_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed-FP32 instructions are disabled for all device code (see DESIGN notes on gfx950).
# Code object v5 so that the HIP runtime bundled with PyTorch (ROCm 7.0) loads it too.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-mcode-object-version=5",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall", "-Werror", *DEVICE_FLAGS,
           "-I", os.path.join(ROOT, "include"),
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed with status {r.returncode}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
