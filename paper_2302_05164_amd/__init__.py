"""MI355X-native matrix-free thermal model of laser powder-bed fusion.

The computation lives in libpbftherm.so (HIP kernels for gfx950 behind the C ABI
declared in include/pbftherm.h); `pbftherm` is the Python binding.
"""
from . import pbftherm  # noqa: F401
from .pbftherm import PREC_FP32, PREC_FP64, PbfError, Simulation, from_problem  # noqa: F401
