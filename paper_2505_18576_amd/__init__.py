"""MI355X-native AMG with filtering (AMGF) for interior-point contact Schur systems.

The solver lives in ``libamgf.so`` (HIP kernels for gfx950 behind the C ABI of
include/amgf.h); ``paper_2505_18576_amd.amgf`` is its ctypes binding.
"""
from .amgf import AMGF, AMGFError, default_options, load_library, SolveInfo  # noqa: F401
