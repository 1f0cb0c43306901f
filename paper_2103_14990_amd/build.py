"""Builds libdlmpc.so in-tree for gfx950 with hipcc (``python -m paper_2103_14990_amd.build``).

Each source is compiled to its own object in parallel, then the objects are linked.
``incremental=True`` (``--incremental``) keeps objects newer than their source and every
header; the default recompiles everything.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
OBJDIR = os.path.join(LIBDIR, "obj")
LIB = os.path.join(LIBDIR, "libdlmpc.so")
SOURCES = ["setup_host.cpp", "setup_kernels.hip", "admm_kernels.hip", "batch_kernels.hip",
           "warmstart_kernels.hip", "dlmpc_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed-FP32 instructions are disabled for all device code (see DESIGN notes on gfx950).
# Code object v5 so that the HIP runtime bundled with PyTorch (ROCm 7.0) loads it too.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-mcode-object-version=5",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Werror"]


def _headers():
    return glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(ROOT, "include", "*.h"))


def _compile(src, obj, verbose):
    cmd = [HIPCC, *COMMON, *DEVICE_FLAGS,
           "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, src), "-o", obj + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        return f"{src}:\n{r.stdout}{r.stderr}"
    os.replace(obj + ".tmp", obj)
    return None


def build(verbose: bool = False, incremental: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    newest_header = max(os.path.getmtime(h) for h in _headers())
    todo, objs = [], []
    for s in SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o")
        objs.append(obj)
        if incremental and os.path.exists(obj):
            t = os.path.getmtime(obj)
            if t > os.path.getmtime(os.path.join(CSRC, s)) and t > newest_header:
                continue
        todo.append((s, obj))
    with ThreadPoolExecutor(max_workers=jobs or min(len(SOURCES), os.cpu_count() or 1)) as ex:
        errs = [e for e in ex.map(lambda so: _compile(*so, verbose), todo) if e]
    if errs:
        sys.stderr.write("\n".join(errs))
        raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *COMMON, *DEVICE_FLAGS, "-shared", *objs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"link failed with status {r.returncode}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
