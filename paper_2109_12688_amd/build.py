"""Builds the gfx950 shared library libnadmm.so in-tree with hipcc.

Usage:  python -m paper_2109_12688_amd.build      (or build() from Python)
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libnadmm.so")
SOURCES = ["kernels.hip", "adjoint.hip", "reduce.hip", "capi.hip", "noalloc.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # packed fp32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def source_files() -> list:
    """Every file the library is compiled from: the HIP sources and headers
    of csrc/ and the public header."""
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                   if f.endswith((".hip", ".h")))
    return files + [os.path.join(ROOT, "include", "nadmm.h")]


def sources_digest() -> str:
    """SHA-256 over the names and contents of source_files(); compiled into
    the library (nadmm_source_digest) so that a stale build is detected."""
    h = hashlib.sha256()
    for path in source_files():
        h.update(os.path.basename(path).encode() + b"\0")
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; the ROCm toolchain is required to build libnadmm.so")
    return exe


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libnadmm.so (always rebuilds)."""
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), *HIPCC_FLAGS, f'-DNADMM_SOURCE_DIGEST="{sources_digest()}"',
           "-I", os.path.join(ROOT, "include"),
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stderr[-8000:]}")
    if verbose:
        noise = "is not a recognized feature for this target"
        for line in res.stderr.splitlines():
            if noise not in line:
                print(line)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
