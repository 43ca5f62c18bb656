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
    # host code: only the C ABI (declared with default visibility in
    # include/nadmm.h) is exported from the shared library
    "-Xarch_host", "-fvisibility=hidden",
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


# Host-code sanitizers (address, undefined behaviour) for a checking build;
# the device code is built as usual.
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """Path of the address-sanitizer runtime that a process loading a
    sanitized build must preload."""
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "lib", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = shutil.which("clang") or "/opt/rocm/llvm/bin/clang"
    res = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return res.stdout.strip()


def build(verbose: bool = False, out: str = LIB, sanitize: bool = False) -> str:
    """Compile every HIP source into `out` (libnadmm.so in the package by
    default; always rebuilds).  sanitize: host code with ASan and UBSan."""
    tmp = out + f".tmp{os.getpid()}"
    cmd = [hipcc(), *HIPCC_FLAGS, *(SANITIZE_FLAGS if sanitize else []),
           f'-DNADMM_SOURCE_DIGEST="{sources_digest()}"',
           "-I", os.path.join(ROOT, "include"),
           # only the C ABI is exported (kernel stubs and C++ helpers stay local)
           "-Wl,--version-script=" + os.path.join(CSRC, "exports.map"),
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
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
