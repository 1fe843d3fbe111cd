"""MI355X-native warm-started stochastic reconfiguration (WSSR) step.

The computation lives in libwssr.so (HIP kernels for gfx950, C ABI in
include/wssr.h); `wssr.Wssr` is its Python binding.
"""
from .wssr import Wssr, WssrError, lib, version  # noqa: F401
