"""MI355X-native differentiable tile-based Gaussian rasterizer (gfx950 HIP).

Hot path of Mini-Splatting2-style scene modelling (arXiv 2411.12788) behind the
C ABI in include/msplat.h; this package is its Python binding:
  raster    -- per-stage calls (project, bin, render_forward/backward, ...)
  autograd  -- torch.autograd.Function with recompute-in-backward
  serve     -- continuous-batching novel-view server
"""
from . import _lib  # noqa: F401

__all__ = ["raster", "autograd", "serve"]
