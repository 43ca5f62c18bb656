"""FP64 CPU oracle for Nesterov-accelerated ADMM diffeomorphic registration.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library.
"""
from .nadmm_ref import *  # noqa: F401,F403
