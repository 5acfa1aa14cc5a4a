"""Build libsgn.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2306_09731_amd.build

Each source is compiled to an object in parallel, then linked into
paper_2306_09731_amd/libsgn.so.  Every build recompiles.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsgn.so")
BUILD_DIR = os.path.join(PKG, "_build")

# (source, object name, extra flags): the kernels are compiled once per
# working precision into their own namespaces.
SOURCES = [
    ("sgn_kernels.hip", "sgn_kernels_fp64", ["-DSGN_PREC=64"]),
    ("sgn_kernels.hip", "sgn_kernels_fp32", ["-DSGN_PREC=32"]),
    ("sgn_dispatch.cpp", "sgn_dispatch", []),
    ("sgn_cnn.hip", "sgn_cnn", []),
    ("sgn_refine.hip", "sgn_refine", []),
    ("sgn_noalloc.hip", "sgn_noalloc", []),
    ("sgn_fgmres.hip", "sgn_fgmres", []),
    ("sgn_api.cpp", "sgn_api", []),
]

# Packed FP32 instructions are disabled for all device code.
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libsgn")
    return path


def _compile(item) -> str:
    src, name, extra = item
    obj = os.path.join(BUILD_DIR, name + ".o")
    lang = [] if src.endswith(".hip") else ["-x", "hip"]
    cmd = [hipcc(), *HIP_FLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libsgn.so failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
