"""MI355X (gfx950) Gaussian-splatting rasterizer of RT-GuIDE (arXiv 2409.18122).

The library (librtg.so, built from csrc/ by build.py) exposes the C ABI of
include/rtg.h; ``raster`` wraps it for PyTorch tensors.  Importing the package
does not load the library; ``raster`` functions load it on first use and fail
loudly if it is missing.
"""
from . import _lib  # noqa: F401

__all__ = ["raster", "build"]
