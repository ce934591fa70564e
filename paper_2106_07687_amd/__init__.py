"""MI355X-native DNN-MG hot path: Python side of the C-ABI in include/dnnmg.h.

The numerical work runs in libdnnmg.so (hand-written gfx950 HIP kernels).  This
package holds only the ctypes binding (`_lib`) and the build script (`build`).
"""
from ._lib import (Context, State, Net, Batch, DnnmgError, load, header_symbols, LIB_PATH,
                   oscillation)

__all__ = ["Context", "State", "Net", "Batch", "DnnmgError", "load", "header_symbols", "LIB_PATH",
           "oscillation"]
