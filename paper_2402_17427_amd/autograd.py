"""The rasterizer as a torch.autograd.Function.

VastGaussian (arXiv 2402.17427), section 3: the renderer R(G, C) is
differentiable and each cell's Gaussians are optimised by gradient
descent on an image loss.  `rasterize` renders one view with the HIP
forward (projection, binning, sort, blend) and, on backward, runs the HIP
backward, which by default recomputes the blend state from the stored
final transmittance and last-contributor index (no per-contributor state
is kept).  `RasterSettings(store_state=True)` selects the variant that
keeps (alpha, T) for every evaluated (entry, pixel) from the forward and
reads it in the backward, for memory/time comparison.

Inputs are the activated parameters as [P][N] float32 CUDA planes:
mean [3][N], scale [3][N] (> 0), quat [4][N] (w, x, y, z), opacity [N] in
(0, 1), sh [3K][N] (K = 1, 4, 9 or 16).  Output: image [3][H][W].
"""
from __future__ import annotations

import dataclasses

import torch
from torch.autograd.function import once_differentiable

from .raster import DeviceGaussians, Frame

_DEG = {1: 0, 4: 1, 9: 2, 16: 3}


@dataclasses.dataclass
class RasterSettings:
    cam: object                     # camera (R, t, fx, fy, cx, cy, width, height, near, bg)
    tile: tuple = (16, 16)
    store_state: bool = False


class RasterizeFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, settings: RasterSettings, mean, scale, quat, opacity, sh):
        K = sh.shape[0] // 3
        if K not in _DEG or sh.shape[0] != 3 * K:
            raise ValueError(f"sh must have 3K rows with K in {sorted(_DEG)}, got {tuple(sh.shape)}")
        g = DeviceGaussians(mean.detach().contiguous(), scale.detach().contiguous(), quat.detach().contiguous(),
                            opacity.detach().contiguous(), sh.detach().contiguous(), _DEG[K])
        f = Frame(g.n, g.sh_degree, settings.cam, settings.tile, device=mean.device)
        f.ensure_capacity(g)
        state = None
        if settings.store_state:
            state = torch.empty(max(f.state_bytes(), 1), dtype=torch.uint8, device=mean.device)
            f.render_fwd_stored(state)
        else:
            f.render_fwd()
        f.check_status()
        ctx.frame, ctx.g, ctx.state = f, g, state
        return f.image

    @staticmethod
    @once_differentiable
    def backward(ctx, dimg):
        f, g = ctx.frame, ctx.g
        d = dimg.contiguous().float()
        if ctx.state is not None:
            f.render_bwd_stored(g, d, ctx.state)
        else:
            f.render_bwd(g, d)
        gr = f.grads()
        ctx.frame = ctx.g = ctx.state = None
        return None, gr["mean"], gr["scale"], gr["quat"], gr["opacity"], gr["sh"]


def rasterize(mean, scale, quat, opacity, sh, settings: RasterSettings) -> torch.Tensor:
    """Differentiable render of one view: image [3][H][W]."""
    return RasterizeFunction.apply(settings, mean, scale, quat, opacity, sh)
