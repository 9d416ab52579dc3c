"""MI355X map-making: PCG with block-diagonal and two-level preconditioners
(Puglisi et al. 2018) behind the C ABI of include/mapmaker.h.

``mapmaker`` is the thin ctypes binding; ``build`` compiles libmapmaker.so.
"""
from . import mapmaker  # noqa: F401
from .mapmaker import (Context, MapmakerError, F32, F64, NOISE_AUTO, NOISE_DIRECT,  # noqa: F401
                       NOISE_FFT)
