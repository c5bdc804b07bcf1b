"""MI355X (gfx950) quasi-cylindrical arbitrary-order PSATD particle-in-cell cycle.

The compute path is the HIP library libpic.so (csrc/, C interface in
include/pic.h); `pic` is its thin Python binding.
"""
from .pic import (Simulation, PicError, load, fft_z, dht_gemm, batch_step, Batch, COMP, H_FP32, H_BF16X3, H_FP16X3,
                  KPERP_J0_ZEROS, KPERP_SINE, KPERP_JM_ZEROS, EXPORTED, LIB_PATH)

__all__ = ["Simulation", "PicError", "load", "fft_z", "dht_gemm", "batch_step", "Batch", "COMP", "H_FP32", "H_BF16X3",
           "H_FP16X3", "KPERP_J0_ZEROS", "KPERP_SINE", "KPERP_JM_ZEROS", "EXPORTED", "LIB_PATH"]
