"""MI355X-native differentiable rasterizer for generalized-exponential splats.

Implements the rendering hot path of DyGASR (arXiv 2411.09156): projection of
GES splats (Sec. 3.2, Eq. 3-7), tile binning by a radix sort on
(tile | depth) keys, front-to-back compositing (Eq. 5) and the hand-written
adjoint, all as HIP kernels for gfx950 behind the C ABI in include/gesr.h.
"""
from .drt import drt_scale  # noqa: F401
from .rasterizer import GESRender, Rasterizer, RasterSettings, Splats, render  # noqa: F401
