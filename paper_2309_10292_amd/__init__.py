"""MI355X-native Gray-Scott 7-point-stencil step (HIP for gfx950 behind a C ABI).

`gs` is the ctypes binding of libgs.so (include/gs.h). Importing the package
touches neither the GPU nor the library; the first call loads libgs.so and
raises if it has not been built.
"""
from . import gs  # noqa: F401

__all__ = ["gs"]
