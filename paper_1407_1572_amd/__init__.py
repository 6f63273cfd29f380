"""MI355X (gfx950) Inverse Fast Multipole Method: FP64 factor + solve.

The numerical work runs in ``libifmm.so`` (HIP kernels + C-ABI, see
include/ifmm.h); ``IFMMSolver`` is the Python face of that ABI.
"""
from .ifmm import IFMMError, IFMMSolver, LIB_PATH, load  # noqa: F401
