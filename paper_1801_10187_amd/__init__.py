"""SRD multiparticle collision dynamics on one AMD MI355X (gfx950).

The hot path lives in libmpcd.so (HIP kernels behind the C ABI of
include/mpcd.h); `binding` marshals arguments to it with ctypes, and
`serve` runs many independent simulations concurrently on the device.
"""
from .binding import (AT, FP32, FP64, SRD, Batch, MpcdError, Sim, copy_kernel,
                      declared_symbols, load, make_params, philox)

__all__ = ["AT", "FP32", "FP64", "SRD", "Batch", "MpcdError", "Sim", "copy_kernel",
           "declared_symbols", "load", "make_params", "philox"]
