"""MI355X-native TVB-AdEx parameter-sweep engine (arXiv:2311.13337 hot path).

The compute path is libvadx.so (HIP kernels for gfx950 behind the C ABI in
include/vadx.h); ``vadx`` is its ctypes binding and ``inputs`` the seeded
synthetic workloads.
"""
__all__ = ["inputs", "vadx", "build"]
