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

Steady state: the buffers of a view (projection, bins, workspaces, image)
come from a pool keyed by the view's shape and reused across steps, so a
training step allocates only the gradient tensors (from PyTorch's caching
allocator) and reads nothing back from the device.  The pair count stays
on the device; it is copied asynchronously to pinned host memory after
each forward, and the next forward on the same buffers grows them ahead of
need when the last count came within 20 % of the capacity.  A view whose
pairs overflowed the capacity anyway renders NaN (and its backward leaves
zero gradients); the next forward on those buffers reports it with a
warning and grows them.
"""
from __future__ import annotations

import dataclasses
import math
import warnings
import weakref

import torch
from torch.autograd.function import once_differentiable

from . import _native as N
from .raster import SH_DIM, DeviceGaussians, Frame

_DEG = {1: 0, 4: 1, 9: 2, 16: 3}
_GROW_AT = 0.8       # grow when the last pair count exceeded this fraction of the capacity
_HEADROOM = 1.5      # new capacity = headroom x the last pair count


@dataclasses.dataclass
class RasterSettings:
    cam: object                     # camera (R, t, fx, fy, cx, cy, width, height, near, bg)
    tile: tuple = (16, 16)
    store_state: bool = False


class _Token:
    """Alive while an autograd context still needs the buffers it rendered with."""


class _Slot:
    def __init__(self, frame: Frame):
        self.frame = frame
        self.state = None
        self.ctx_ref = None            # weakref to the _Token of the pending backward
        self.out_ref = None            # weakref to the returned image view
        self.host = torch.zeros(2, dtype=torch.int32).pin_memory()   # (status, pairs needed)
        self.event = None
        self.checked = True

    def free(self) -> bool:
        return (self.ctx_ref is None or self.ctx_ref() is None) and (self.out_ref is None or self.out_ref() is None)


_pool: dict = {}


def _key(g: DeviceGaussians, st: RasterSettings, device):
    c = st.cam
    return (str(device), g.n, g.sh_degree, int(c.width), int(c.height), tuple(st.tile))


def _acquire(g: DeviceGaussians, st: RasterSettings, device) -> _Slot:
    slots = _pool.setdefault(_key(g, st, device), [])
    for s in slots:
        if s.free():
            return s
    # a new set of buffers for this view shape: size the pair buffers once
    # (the only host read, on first use)
    f = Frame(g.n, g.sh_degree, st.cam, st.tile, device=device)
    f.ensure_capacity(g)
    need = f.pairs()[1]
    f.set_capacity(max(int(math.ceil(need * _HEADROOM)) + 1024, f.capacity))
    s = _Slot(f)
    slots.append(s)
    return s


def _check_previous(s: _Slot):
    """Inspect the pair count of the last forward on these buffers if the
    device has produced it already (no wait), and grow them ahead of need."""
    if s.checked or s.event is None or not s.event.query():
        return
    s.checked = True
    status, need = int(s.host[0]), int(s.host[1])
    f = s.frame
    if status == N.GS_ERR_CAPACITY:
        warnings.warn(f"rasterize: the previous view needed {need} pairs, more than the capacity {f.capacity}; "
                      f"its image was NaN and its gradients zero; growing the buffers", RuntimeWarning)
    if need > _GROW_AT * f.capacity:
        f.set_capacity(int(math.ceil(need * _HEADROOM)) + 1024)
        s.state = None


class RasterizeFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, settings: RasterSettings, mean, scale, quat, opacity, sh):
        K = sh.shape[0] // 3
        if K not in _DEG or sh.shape[0] != 3 * K:
            raise ValueError(f"sh must have 3K rows with K in {sorted(_DEG)}, got {tuple(sh.shape)}")
        g = DeviceGaussians(mean.detach().contiguous(), scale.detach().contiguous(), quat.detach().contiguous(),
                            opacity.detach().contiguous(), sh.detach().contiguous(), _DEG[K])
        s = _acquire(g, settings, mean.device)
        _check_previous(s)
        f = s.frame
        f.cam = settings.cam
        f.c_cam = N.make_camera(settings.cam)
        f.project(g)
        f.bin_sort()
        if settings.store_state:
            nb = max(f.state_bytes(), 1)
            if s.state is None or s.state.numel() < nb:
                s.state = torch.empty(nb, dtype=torch.uint8, device=mean.device)
            f.render_fwd_stored(s.state)
        else:
            f.render_fwd()
        # the status and the pairs the view needed, to pinned host memory
        s.host[0:1].copy_(f.status, non_blocking=True)
        s.host[1:2].copy_(f.pair_count[1:2], non_blocking=True)
        if s.event is None:
            s.event = torch.cuda.Event()
        s.event.record()
        s.checked = False
        token = _Token()
        out = f.image.view_as(f.image)
        s.ctx_ref, s.out_ref = weakref.ref(token), weakref.ref(out)
        ctx.slot, ctx.g, ctx.token, ctx.store = s, g, token, settings.store_state
        return out

    @staticmethod
    @once_differentiable
    def backward(ctx, dimg):
        s, g = ctx.slot, ctx.g
        f = s.frame
        d = dimg.contiguous().float()
        n, dev = g.n, d.device
        K = SH_DIM[g.sh_degree]
        out = dict(mean=torch.empty((3, n), device=dev), scale=torch.empty((3, n), device=dev),
                   quat=torch.empty((4, n), device=dev), opacity=torch.empty(n, device=dev),
                   sh=torch.empty((3 * K, n), device=dev))
        if ctx.store:
            f.render_bwd_stored(g, d, s.state, out=out)
        else:
            f.render_bwd(g, d, out=out)
        ctx.slot = ctx.g = ctx.token = None
        return None, out["mean"], out["scale"], out["quat"], out["opacity"], out["sh"]


def rasterize(mean, scale, quat, opacity, sh, settings: RasterSettings) -> torch.Tensor:
    """Differentiable render of one view: image [3][H][W]."""
    return RasterizeFunction.apply(settings, mean, scale, quat, opacity, sh)


def held_bytes(settings: RasterSettings, g: DeviceGaussians) -> dict:
    """Device bytes the pooled buffers of a view shape hold between forward
    and backward: the frame's buffers, and the stored blend state when
    `settings.store_state` (for the recompute-vs-stored comparison)."""
    slots = _pool.get(_key(g, settings, g.mean.device), [])
    if not slots:
        return {"frame": 0, "state": 0}
    s = slots[0]
    f = s.frame
    tensors = [f.rec, f.depth, f.rect, f.tiles_touched, f.first, f.ranges, f.tile_order, f.pair_count, f.status, f.image,
               f.final_T, f.n_contrib, f.keys, f.vals, f.ws, f.bwd_ws, f.masks, f.grad2d]
    fb = sum(t.numel() * t.element_size() for t in tensors if t is not None)
    sb = s.state.numel() if (settings.store_state and s.state is not None) else 0
    return {"frame": int(fb), "state": int(sb)}
