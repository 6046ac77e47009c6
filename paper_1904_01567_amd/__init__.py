"""MI355X-native gMCO hot path: batched L-BFGS dwell-time optimisation of
many HDR brachytherapy plans at once (arXiv 1904.01567), as hand-written HIP
for gfx950 behind the C-ABI of include/gmco.h.

There is no CPU fallback: without the built library (libgmco.so) and a
gfx950 GPU every call raises.
"""
from ._binding import (DTYPES, EXPORTS, GmcoError, Network, Planner,  # noqa: F401
                       STATUS_NAMES, load_library, LIB_PATH, optimize_many)

__all__ = ["Planner", "Network", "GmcoError", "load_library", "DTYPES", "STATUS_NAMES",
           "EXPORTS", "LIB_PATH", "optimize_many"]
