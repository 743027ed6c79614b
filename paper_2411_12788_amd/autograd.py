"""torch.autograd.Function around the C ABI, with recompute in backward.

Forward runs projection, binning, sort and compositing for all V views in one
launch per stage and keeps only the inputs plus 8 bytes per pixel (T_final and
the list position of the last included Gaussian).  Backward recomputes the
projection and the sorted lists — both are deterministic, so they come out
bit-identical to the forward's — and then runs the masked pixel backward and
the projection backward.  With ``save_lists=True`` the forward's records and
lists are kept instead (more memory, no recompute); both modes run the same
kernels on bit-identical lists, so their gradients differ only by the
summation order of the float atomics that gather per-pixel partials
(~1e-6 relative); with ``deterministic=True`` the pixel backward uses the
library's ordered reduction instead and the two modes agree bitwise.

Differentiable output: colour [3, P].  Depth and the argmax index are marked
non-differentiable; per-Gaussian accumulations, when requested, are returned
through the ``accum`` dict and are not part of the graph.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import torch

from . import raster as R


class RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means, scales, quats, opacity, sh, cams, opts, sh_degree, active, save_lists, accum,
                deterministic):
        scene = R.DeviceScene(means.contiguous(), scales.contiguous(), quats.contiguous(), opacity.contiguous(),
                              sh.contiguous(), int(sh_degree))
        proj = R.project(scene, cams, opts)
        binned = R.bin(proj, cams, scene.n)
        frame = R.render_forward(scene, proj, binned, cams, opts, accum=accum, extras=False)
        ctx.cams, ctx.opts, ctx.sh_degree = cams, opts, int(sh_degree)
        ctx.active = active
        ctx.deterministic = bool(deterministic)
        ctx.lists = (proj, binned) if save_lists else None
        ctx.save_for_backward(scene.means, scene.scales, scene.quats, scene.opacity, scene.sh, frame.t_final,
                              frame.last)
        ctx.mark_non_differentiable(frame.depth, frame.imax)
        return frame.color, frame.depth, frame.imax

    @staticmethod
    def backward(ctx, dcolor, ddepth, dimax):
        means, scales, quats, opacity, sh, t_final, last = ctx.saved_tensors
        scene = R.DeviceScene(means, scales, quats, opacity, sh, ctx.sh_degree)
        if ctx.lists is not None:
            proj, binned = ctx.lists
        else:
            proj = R.project(scene, ctx.cams, ctx.opts)
            binned = R.bin(proj, ctx.cams, scene.n)
        frame = R.Frame(None, None, None, t_final, last, None, None)
        grads, _ = R.render_backward(scene, proj, binned, ctx.cams, ctx.opts, frame, dcolor.contiguous(),
                                     ctx.active, deterministic=ctx.deterministic)
        ctx.lists = None
        return (grads["means"], grads["scales"], grads["quats"], grads["opacity"], grads["sh"],
                None, None, None, None, None, None, None)


def rasterize(means: torch.Tensor, scales: torch.Tensor, quats: torch.Tensor, opacity: torch.Tensor,
              sh: torch.Tensor, cams: Sequence, opts: Optional[R.RasterOpts] = None, sh_degree: int = 3,
              active: Optional[torch.Tensor] = None, save_lists: bool = False,
              accum: Optional[Dict[str, torch.Tensor]] = None, deterministic: bool = False):
    """Differentiable render of V views.  Layouts as in ``raster.DeviceScene``
    (means [3,n], scales [3,n], quats [4,n], opacity [n], sh [16,3,n]; activated
    scales and opacity).  Returns colour [3, P], depth [P], imax [P] with P the
    total pixel count (views concatenated, row-major within a view)."""
    opts = opts or R.RasterOpts()
    return RasterizeFn.apply(means, scales, quats, opacity, sh, list(cams), opts, sh_degree, active, save_lists,
                             accum, deterministic)


def split_views(x: torch.Tensor, cams: Sequence):
    """Split a [..., P] per-pixel tensor into per-view [..., H, W] tensors."""
    out, off = [], 0
    for c in cams:
        m = int(c.width) * int(c.height)
        out.append(x[..., off:off + m].reshape(*x.shape[:-1], int(c.height), int(c.width)))
        off += m
    return out
