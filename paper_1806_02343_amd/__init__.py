"""gfx950 DG ideal-MHD library: thin Python binding of libdgmhd.so.

The binding only marshals arguments: every step of the scheme runs in the HIP
kernels behind the C ABI declared in include/dg.h.  PyTorch provides device
memory and the stream.  If the compiled library is missing, importing the
binding raises; there is no fallback path.
"""
from .binding import (DG, DGError, DGWarning, DG_FP32, DG_FP64, DG_GLM, DG_POWELL, DG_LIM_CHAR, DG_LIM_LEARNED,
                      DG_LIM_POS, DG_LIM_TVB, LIB_PATH, load_library)

__all__ = ["DG", "DGError", "DGWarning", "DG_FP32", "DG_FP64", "DG_GLM", "DG_POWELL", "DG_LIM_TVB", "DG_LIM_CHAR",
           "DG_LIM_POS", "DG_LIM_LEARNED", "LIB_PATH", "load_library"]
