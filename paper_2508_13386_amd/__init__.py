"""MI355X multilevel elastodynamics timestep library (HIP, gfx950).

The native library libms.so (built from csrc/ by `build.py`) implements the
hot path; `ms` is its ctypes binding.
"""
from . import ms  # noqa: F401

__all__ = ["ms"]
