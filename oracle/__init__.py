"""FP64 CPU oracle for SA-AMG-PCG and its adjoint.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP library and never imports it.
"""
from .oracle import *  # noqa: F401,F403
