"""MI355X (gfx950) hot path of N^5 excited-state-specific MP2 (ESMP2-TOP(1) and TOP(k)).

Thin Python binding of the C ABI in include/esmp2.h: argument marshalling
only.  Every step of the computation runs in the HIP kernels of
libesmp2.so; importing this package fails loudly when the library has not
been built.  PyTorch supplies device memory and the stream.
"""
from ._lib import (ESMP2_OK, ESMP2_INVALID_ARG, ESMP2_BAD_ORDER, ESMP2_NOT_SPD,  # noqa: F401
                   ESMP2_NOT_CONVERGED, ESMP2_OOM, ESMP2_HIP_ERROR, ESMP2_UNSUPPORTED,
                   ESMP2_FP64, ESMP2_FP32, ESMP2_BF16, ESMP2_BASIS_TOP, ESMP2_BASIS_SEMICANONICAL, Esmp2Error,
                   Handle, lib, LIB_PATH, solve_batch, large_top_count)
from .autograd import e2_top  # noqa: F401,E402
