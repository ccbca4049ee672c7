"""dgj: implicit DG compressible Navier-Stokes hot path (arxiv 2002.04222)
on AMD MI355X.

The compute runs in the HIP library lib/libdgj.so (C ABI declared in
include/dgj.h); this package only marshals arguments to it.  There is no
CPU fallback: importing the binding fails loudly when the library is
missing.
"""
from .binding import (Batch, Context, DgjError, load_library, DGJ_OK, DGJ_PC_F64, DGJ_PC_F32,  # noqa: F401
                      DGJ_PC_BF16, DGJ_SDIRK2, DGJ_SDIRK3, LIB_PATH)
