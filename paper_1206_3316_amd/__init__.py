"""MI355X-native linearized deviational phonon Monte Carlo.

The compute path is the HIP library ``libdmc.so`` (built from ``csrc/`` for
gfx950) behind the C ABI of ``include/dmc.h``; ``binding`` is its ctypes
binding.  Importing this package does not load the library; the first call
does, and fails loudly if it was not built.
"""
from . import binding  # noqa: F401
from .binding import Material, Result, simulate  # noqa: F401

__all__ = ["binding", "Material", "Result", "simulate"]
