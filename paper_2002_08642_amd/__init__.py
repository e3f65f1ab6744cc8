"""MI355X-native penalized pseudo-spectral Navier-Stokes step (gfx950, HIP).

The compute path is the C-ABI library ``libfsi.so`` (declared in
``include/fsi.h``); ``fsi`` is its ctypes binding.
"""

from .fsi import Solver, FsiError, load_library, plate_pose, PROFILE_COS, PROFILE_TANH, PREC_FP32, PREC_FP64  # noqa: F401
