"""MI355X-native differentiable Gaussian tile rasterizer (gfx950, HIP).

The hot path of VastGaussian's per-cell 3D Gaussian Splatting optimisation
(arXiv 2402.17427, section 3): EWA projection with SH colour, tile binning
and radix sort, front-to-back alpha blending and its backward pass, all as
hand-written HIP kernels behind the C ABI in include/gs.h.  This package is
the thin Python binding (ctypes) plus torch glue for buffers and streams.
"""
from . import _native  # noqa: F401

__all__ = ["_native"]
