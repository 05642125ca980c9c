"""V-family Mersenne Twister generators (arXiv 2309.16682) on MI355X.

The hot path lives in libvmt.so (HIP kernels for gfx950 behind the C ABI of
include/vmt.h); `vmt` is its thin ctypes binding.
"""
from . import vmt  # noqa: F401

__all__ = ["vmt"]
