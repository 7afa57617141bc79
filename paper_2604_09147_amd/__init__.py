"""Adaptive mixed-precision H_h matrices on AMD MI355X (gfx950).

The native library (lib/libhhmat.so, built from csrc/) does all the work; this
package only marshals arguments. See include/hh.h for the C ABI."""
from .hh import (HMatrix, HHError, plan, quantize, quantize_cont, matvec_batch, lib, LIB_PATH,  # noqa: F401
                 switch_level_search,
                 LOG, INV_R, INV_R2, GAUSS, MATERN, DOUBLE_LAYER,
                 FMT_FP64, FMT_FP32, FMT_FP16, FMT_BF16, FMT_CONT, FMT_Q43)
