"""MI355X (gfx950) Nesterov-accelerated ADMM diffeomorphic registration.

The compute path is the HIP library libnadmm.so (C ABI in include/nadmm.h).
``paper_2109_12688_amd.api`` marshals torch tensors into it; ``_lib`` holds
the ctypes binding.
"""
from ._lib import EXPORTS, NadmmError, load  # noqa: F401

__all__ = ["EXPORTS", "NadmmError", "load"]
