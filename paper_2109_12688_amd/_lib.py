"""ctypes binding of libnadmm.so (the C ABI declared in include/nadmm.h).

Argument marshalling only: every step of the registration path runs in the
library's HIP kernels.  Tensors are torch tensors on the ROCm ("cuda")
device; work is enqueued on torch's current stream.  There is no CPU
fallback: if the library is missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# NADMM_LIBRARY selects another build of the same sources (the sanitized
# build of the host-code checks); it must carry the same source digest.
LIB_PATH = os.environ.get("NADMM_LIBRARY") or os.path.join(PKG, "libnadmm.so")

NADMM_OK = 0
STATUS_NAMES = {0: "NADMM_OK", 1: "NADMM_ERR_INVALID_ARG", 2: "NADMM_ERR_UNSUPPORTED_SIZE",
                3: "NADMM_ERR_WORKSPACE", 4: "NADMM_ERR_HIP", 5: "NADMM_ERR_NONFINITE",
                6: "NADMM_ERR_DIVERGED"}
CHECK_FINITE, CHECK_DIVERGENCE = 1, 2


class Dims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("theta", ctypes.c_double),
                ("order", ctypes.c_int32), ("data_term", ctypes.c_int32),
                ("eps", ctypes.c_double), ("outer", ctypes.c_int32), ("iters", ctypes.c_int32)]


class Pyramid(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("outer", ctypes.c_int32 * 4), ("iters", ctypes.c_int32 * 4)]


class NadmmError(RuntimeError):
    def __init__(self, fn: str, status: int, detail: str):
        self.status = status
        super().__init__(f"{fn}: {STATUS_NAMES.get(status, status)}: {detail}")


_P = ctypes.c_void_p
_SIGS = {
    "nadmm_abi_version": ([], ctypes.c_int),
    "nadmm_source_digest": ([], ctypes.c_char_p),
    "nadmm_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "nadmm_last_error": ([], ctypes.c_char_p),
    "nadmm_workspace_size": ([Dims, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "nadmm_register_threshold": ([Dims, ctypes.POINTER(Params), ctypes.c_double, ctypes.c_double, _P, _P, _P,
                                  _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "nadmm_register": ([Dims, ctypes.POINTER(Params), _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P],
                       ctypes.c_int),
    "nadmm_register_checked": ([Dims, ctypes.POINTER(Params), ctypes.c_uint32, _P, _P, _P, _P, _P, _P, _P,
                                ctypes.c_size_t, _P], ctypes.c_int),
    "nadmm_register_bf16": ([Dims, ctypes.POINTER(Params), _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t,
                             _P], ctypes.c_int),
    "nadmm_workspace_size_batch": ([Dims, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "nadmm_register_batch": ([Dims, ctypes.c_int32, ctypes.POINTER(Params), _P, _P, _P, _P, _P, _P,
                              ctypes.c_size_t, _P], ctypes.c_int),
    "nadmm_workspace_size_mixed": ([ctypes.c_int32, ctypes.POINTER(Dims), ctypes.POINTER(ctypes.c_size_t)],
                                   ctypes.c_int),
    "nadmm_register_mixed": ([ctypes.c_int32, ctypes.POINTER(Dims), ctypes.POINTER(Params), _P, _P, _P, _P, _P,
                              ctypes.c_size_t, _P], ctypes.c_int),
    "nadmm_workspace_size_grad": ([Dims, ctypes.POINTER(Params), ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
                                  ctypes.c_int),
    "nadmm_ssd_grad": ([Dims, ctypes.POINTER(Params), ctypes.c_int32, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P],
                       ctypes.c_int),
    "nadmm_autotune": ([Dims, ctypes.c_int32, ctypes.POINTER(Params), _P, ctypes.c_size_t, _P,
                        ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "nadmm_tuned_shapes": ([Dims, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "nadmm_set_shapes": ([Dims, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "nadmm_workspace_size_pyramid": ([Dims, ctypes.POINTER(Pyramid), ctypes.POINTER(ctypes.c_size_t)],
                                     ctypes.c_int),
    "nadmm_register_pyramid": ([Dims, ctypes.POINTER(Params), ctypes.POINTER(Pyramid), _P, _P, _P, _P, _P,
                                ctypes.c_size_t, _P], ctypes.c_int),
    "nadmm_register_pyramid_threshold": ([Dims, ctypes.POINTER(Params), ctypes.POINTER(Pyramid), ctypes.c_double,
                                          ctypes.c_double, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P],
                                         ctypes.c_int),
    "nadmm_admm": ([Dims, ctypes.POINTER(Params), _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "nadmm_fourier_solve": ([Dims, ctypes.POINTER(Params), _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "nadmm_warp": ([Dims, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "nadmm_compose": ([Dims, _P, _P, _P, _P], ctypes.c_int),
    "nadmm_expmap": ([Dims, _P, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "nadmm_jacobian": ([Dims, _P, _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "nadmm_jacobian_noalloc": ([Dims, _P, _P, _P, _P, _P], ctypes.c_int),
    "nadmm_count_nonfinite": ([Dims, _P, ctypes.c_int32, _P, _P], ctypes.c_int),
    "nadmm_profile_enable": ([ctypes.c_int], ctypes.c_int),
    "nadmm_profile_replay": ([Dims, ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_size_t,
                              _P, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "nadmm_profile_read": ([ctypes.c_int, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_int64),
                            ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
}
EXPORTS = tuple(_SIGS)

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libnadmm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2109_12688_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    if path == LIB_PATH:
        from .build import sources_digest
        built, now = lib.nadmm_source_digest().decode(), sources_digest()
        if built != now:
            raise RuntimeError(f"{path} was built from other sources (digest {built[:12]}, sources "
                               f"{now[:12]}): rebuild it with `python -m paper_2109_12688_amd.build`")
    _lib = lib
    return lib


def check(fn: str, status: int) -> None:
    if status != NADMM_OK:
        raise NadmmError(fn, status, load().nadmm_last_error().decode(errors="replace"))


def call(fn: str, *args) -> None:
    check(fn, getattr(load(), fn)(*args))


def profile_enable(on: bool) -> None:
    call("nadmm_profile_enable", 1 if on else 0)


def profile_read() -> dict:
    """{kernel kind: (launches, total ms)} since the previous read (waits for the GPU)."""
    n = 32
    names = (ctypes.c_char_p * n)()
    counts = (ctypes.c_int64 * n)()
    ms = (ctypes.c_double * n)()
    k = load().nadmm_profile_read(n, names, counts, ms)
    if k < 0:
        raise NadmmError("nadmm_profile_read", 4, load().nadmm_last_error().decode(errors="replace"))
    return {names[i].decode(): (int(counts[i]), float(ms[i])) for i in range(k) if counts[i]}
