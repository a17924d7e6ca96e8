"""MI355X-native weighted quadrature (WQ) assembly on unstructured bicubic splines.

The compute path is libwq.so (HIP kernels for gfx950, C ABI in include/wq.h); `wq` is
its ctypes binding.
"""
from . import wq  # noqa: F401
