"""MI355X-native incremental-SVD engine (Brand-style rank-k updates).

The compute path is libisvd.so (hand-written HIP kernels for gfx950 behind a
C ABI, ``include/isvd.h``); ``isvd`` is its thin Python binding.
"""
from .isvd import (Engine, Policy, IsvdError, load_library, EXPORTS, LIB_PATH,
                   ROW, COL, ENTRY, POL_NONE, POL_PERIODIC, POL_ERROR, POL_ANGLE, POL_ADAPTIVE)

__all__ = ["Engine", "Policy", "IsvdError", "load_library", "EXPORTS", "LIB_PATH", "ROW", "COL", "ENTRY",
           "POL_NONE", "POL_PERIODIC", "POL_ERROR", "POL_ANGLE", "POL_ADAPTIVE"]
