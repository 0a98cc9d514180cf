"""MI355X-native HALLaR hot path: HIP kernels behind a C ABI (libhallar.so)
and its ctypes binding.  See include/hallar.h for the ABI."""
from . import hallar  # noqa: F401

__all__ = ["hallar"]
