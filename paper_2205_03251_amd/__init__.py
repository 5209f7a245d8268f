"""gpeval: MI355X-native data-parallel fitness evaluation of tree GP individuals.

The library is libgpeval.so (HIP kernels for gfx950 + host runtime, C ABI in
include/gpeval.h); `gpeval` is its ctypes binding.
"""
from . import gpeval  # noqa: F401
