"""MI355X-native affine-reconstructed nodal DG (aRDG) right-hand side.

The compute path is the HIP library ``libardg.so`` (sources in ``csrc/``,
C ABI in ``include/ardg.h``); ``ardg`` is its ctypes binding and ``build``
compiles it for gfx950.
"""
from . import ardg  # noqa: F401

__all__ = ["ardg"]
