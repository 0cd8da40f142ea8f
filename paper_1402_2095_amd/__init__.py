"""MI355X-native f-thermostat (FTH) hot path.

The compute path lives in ``libfth.so`` (HIP kernels for gfx950 behind the C
ABI of include/fth.h); ``fth`` is its ctypes binding.
"""
from . import fth  # noqa: F401
from .fth import Solver, Server, FthError  # noqa: F401
