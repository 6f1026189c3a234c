"""MI355X-native differentiable Bezier Splatting rasterizer.

The compute path is the C-ABI library ``libbz.so`` (hand-written HIP for
gfx950, declared in ``include/bz.h``); :mod:`paper_2503_16424_amd.bz` is its thin
Python binding.  :mod:`paper_2503_16424_amd.scenes` draws seeded synthetic
inputs.  Importing the package loads nothing; the binding loads the library on
first use and raises if it is missing.
"""
__all__ = ["bz", "scenes"]
