"""MI355X-native radar ray-tracing hot path (trace + FMCW cube synthesis).

The compute lives in libradray.so (hand-written HIP kernels for gfx950,
C ABI in include/radray.h); `binding` is a thin ctypes layer over it.
"""
from .binding import (Context, Batch, RadrayError, load_library, LIB_PATH, EXACT, SEPARABLE,
                      ENGINE_AUTO, DIRECT_FP32, GEMM_BF16X3, GEMM_EXACT, TX_PER_ELEMENT, TX_SHARED, UNIFORM,
                      PROPOSAL, PER_TRIANGLE, KMAX, ALPHA_PER_OBJECT, ALPHA_PER_TRIANGLE)

__all__ = ["Context", "Batch", "RadrayError", "load_library", "LIB_PATH", "EXACT", "SEPARABLE",
           "ENGINE_AUTO", "DIRECT_FP32", "GEMM_BF16X3", "GEMM_EXACT", "TX_PER_ELEMENT", "TX_SHARED", "UNIFORM",
           "PROPOSAL", "PER_TRIANGLE", "KMAX", "ALPHA_PER_OBJECT", "ALPHA_PER_TRIANGLE"]
