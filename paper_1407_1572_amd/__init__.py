"""MI355X (gfx950) Inverse Fast Multipole Method: factor + solve, FP64 or
mixed precision (FP32 factor, FP64 refinement).

The numerical work runs in ``libifmm.so`` (HIP kernels + C-ABI, see
include/ifmm.h); ``IFMMSolver`` is the Python face of that ABI.
"""
from .ifmm import (IFMMError, IFMMSolver, LIB_PATH, factor_batched, load,  # noqa: F401
                   release_cached_memory, solve_batched)
