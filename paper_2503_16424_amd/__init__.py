"""MI355X-native differentiable Bezier Splatting rasterizer.

The compute path is the C-ABI library ``libbz.so`` (hand-written HIP for
gfx950, declared in ``include/bz.h`` and ``include/bz_cnn.h``):

* :mod:`bz` -- thin binding of the rasterizer (sample, bin, forward,
  backward, batches, area order, Xing loss);
* :mod:`optim` -- autograd function and the fitting loop;
* :mod:`graph`, :mod:`autotune` -- a step as one HIP graph replay, launch
  shapes chosen by measurement;
* :mod:`adaptive` -- pruning and densification of curves;
* :mod:`cnn`, :mod:`learned_init` -- the learned curve initialiser on BF16
  matrix-core kernels;
* :mod:`scenes` -- seeded synthetic inputs.

Importing the package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
__all__ = ["bz", "scenes", "optim", "graph", "autotune", "adaptive", "cnn", "learned_init"]
