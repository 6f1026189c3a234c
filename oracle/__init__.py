"""CPU oracle of the Bezier Splatting rasterizer -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  The product (the HIP library and its Python binding) never imports it.
"""
from .oracle import (DEFAULTS, build, chain, forward_backward, lib_path, num_threads,  # noqa: F401
                     render, render_pixels, sample, set_threads, tile_depth)
