"""MI355X-native IFDLBM (arXiv:2306.07603): HIP kernels for gfx950 behind the C ABI of
include/ifdlbm.h, with a ctypes binding of the same names (see ifdlbm.py)."""
from . import workloads  # noqa: F401
from .ifdlbm import *  # noqa: F401,F403
