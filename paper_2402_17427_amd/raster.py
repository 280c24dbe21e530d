"""Torch-facing wrappers of the rasterizer C ABI.

PyTorch supplies device memory and the current HIP stream; every step of
the render (projection, binning, sort, blend, backward) runs in the HIP
kernels behind libgsmi.so.  Nothing here computes on the host besides
buffer sizing.

`Frame` owns every buffer one view needs (so a timed loop allocates
nothing); `render`/`render_backward` are one-shot conveniences.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math

import numpy as np
import torch

from . import _native as N

SH_DIM = {0: 1, 1: 4, 2: 9, 3: 16}


def stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


@dataclasses.dataclass
class DeviceGaussians:
    """Gaussian SoA planes on the GPU (float32): mean [3][N], scale [3][N],
    quat [4][N] (w, x, y, z), opacity [N], sh [3K][N]."""
    mean: torch.Tensor
    scale: torch.Tensor
    quat: torch.Tensor
    opacity: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    @property
    def ld(self) -> int:
        return int(self.mean.stride(0)) if self.mean.dim() == 2 else self.n

    @classmethod
    def from_host(cls, g, device="cuda") -> "DeviceGaussians":
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32)).to(device)
        return cls(f(g.mean), f(g.scale), f(g.quat), f(g.opacity), f(g.sh), int(g.sh_degree))

    def check(self):
        n = self.n
        K = SH_DIM[self.sh_degree]
        for name, t, rows in (("mean", self.mean, 3), ("scale", self.scale, 3), ("quat", self.quat, 4),
                              ("sh", self.sh, 3 * K)):
            if t.dtype != torch.float32 or not t.is_cuda or tuple(t.shape) != (rows, n) or not t.is_contiguous():
                raise ValueError(f"{name}: expected contiguous float32 cuda [{rows}, {n}], got "
                                 f"{t.dtype} {tuple(t.shape)}")
        o = self.opacity
        if o.dtype != torch.float32 or not o.is_cuda or tuple(o.shape) != (n,) or not o.is_contiguous():
            raise ValueError("opacity: expected contiguous float32 cuda [N]")

    def c_struct(self) -> N.gs_gaussians:
        self.check()
        s = N.gs_gaussians()
        s.n = s.ld = self.n
        s.sh_degree = self.sh_degree
        s.mean, s.scale, s.quat = _ptr(self.mean), _ptr(self.scale), _ptr(self.quat)
        s.opacity, s.sh = _ptr(self.opacity), _ptr(self.sh)
        return s


class Frame:
    """All device buffers of one view: projection, bins, image and
    gradients, sized for `n` Gaussians and `capacity` pairs.  Methods
    enqueue on the current torch stream and never synchronise (except
    `ensure_capacity`/`check_status`, which read the device status)."""

    def __init__(self, n: int, sh_degree: int, cam, tile=(16, 16), capacity: int | None = None,
                 device="cuda", grads: bool = True, keep_masks: bool = True, keep_order: bool = True):
        self.n, self.sh_degree, self.device = int(n), int(sh_degree), device
        self.cam = cam
        self.c_cam = N.make_camera(cam)
        self.tile = (int(tile[0]), int(tile[1]))
        self.c_opts = N.make_opts(*self.tile)
        self.W, self.H = int(cam.width), int(cam.height)
        self.ntx = (self.W + self.tile[0] - 1) // self.tile[0]
        self.nty = (self.H + self.tile[1] - 1) // self.tile[1]
        self.n_tiles = self.ntx * self.nty
        n1 = max(self.n, 1)
        self.rec = torch.empty(n1 * N.REC_BYTES // 4, dtype=torch.float32, device=device)
        self.depth = torch.empty(n1, dtype=torch.float32, device=device)
        self.rect = torch.empty(n1 * 4, dtype=torch.int16, device=device)
        self.tiles_touched = torch.empty(n1, dtype=torch.int32, device=device)
        self.first = torch.empty(n1, dtype=torch.int32, device=device)
        self.ranges = torch.empty(self.n_tiles * 2, dtype=torch.int32, device=device)
        # the blend order gs_bin_sort keeps (count, then every tile, longest list first)
        self.tile_order = torch.empty(self.n_tiles + 1, dtype=torch.int32, device=device) if keep_order else None
        self.pair_count = torch.zeros(2, dtype=torch.int32, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        npix = self.W * self.H
        self.image = torch.empty((3, self.H, self.W), dtype=torch.float32, device=device)
        self.final_T = torch.empty((self.H, self.W), dtype=torch.float32, device=device)
        self.n_contrib = torch.empty((self.H, self.W), dtype=torch.int32, device=device)
        K = SH_DIM[self.sh_degree]
        ng = n1 if grads else 1      # forward-only frames keep no gradient planes
        self.g_mean = torch.empty((3, ng), dtype=torch.float32, device=device)
        self.g_scale = torch.empty((3, ng), dtype=torch.float32, device=device)
        self.g_quat = torch.empty((4, ng), dtype=torch.float32, device=device)
        self.g_opacity = torch.empty(ng, dtype=torch.float32, device=device)
        self.g_sh = torch.empty((3 * K, ng), dtype=torch.float32, device=device)
        self.grad2d = torch.empty((9, ng), dtype=torch.float32, device=device)
        self.has_grads = grads
        # the forward keeps its cell masks for the backward (gradient frames)
        self.keep_masks = bool(grads and keep_masks)
        self.capacity = 0
        self.keys = self.vals = self.ws = self.bwd_ws = self.masks = None
        self.set_capacity(capacity if capacity is not None else max(2 * self.n, 1 << 16))
        del npix

    # -- buffers ------------------------------------------------------------
    def set_capacity(self, cap: int):
        cap = int(min(max(cap, 1), (1 << 30) - 1))
        if cap == self.capacity:
            return
        self.capacity = cap
        self.keys = torch.empty(cap, dtype=torch.int64, device=self.device)
        self.vals = torch.empty(cap, dtype=torch.int32, device=self.device)
        nbytes = C.c_size_t(0)
        N.call("gs_bin_sort_workspace", self.n, cap, self.n_tiles, C.byref(nbytes))
        self.ws = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=self.device)
        if self.has_grads:
            N.call("gs_render_bwd_workspace", C.byref(self.c_bins()), C.byref(nbytes))
            # float32 storage keeps the 16-byte alignment the ABI asks for
            self.bwd_ws = torch.empty(max((int(nbytes.value) + 15) // 16 * 4, 4), dtype=torch.float32,
                                      device=self.device)
        if self.keep_masks:
            self.masks = None
            N.call("gs_render_mask_bytes", C.byref(self.c_bins()), C.byref(self.c_opts), C.byref(nbytes))
            self.masks = torch.empty(max(int(nbytes.value) // 8, 1), dtype=torch.int64, device=self.device)

    def c_proj(self) -> N.gs_proj:
        p = N.gs_proj()
        p.rec, p.depth, p.rect, p.tiles_touched = (_ptr(self.rec), _ptr(self.depth), _ptr(self.rect),
                                                   _ptr(self.tiles_touched))
        return p

    def c_bins(self) -> N.gs_bins:
        b = N.gs_bins()
        b.keys, b.vals, b.ranges = _ptr(self.keys), _ptr(self.vals), _ptr(self.ranges)
        b.first = _ptr(self.first)
        b.pair_count, b.status = _ptr(self.pair_count), _ptr(self.status)
        b.pair_capacity = self.capacity
        b.cell_masks = _ptr(self.masks) if self.masks is not None else None
        b.tile_order = _ptr(self.tile_order) if self.tile_order is not None else None
        return b

    def c_grads(self, out: dict | None = None) -> N.gs_grads:
        """Gradient planes: the frame's own, or the caller's `out` (mean,
        scale, quat, opacity, sh: contiguous float32 [P][n] / [n])."""
        g = N.gs_grads()
        if out is None:
            g.ld = max(self.n, 1)
            g.mean, g.scale, g.quat = _ptr(self.g_mean), _ptr(self.g_scale), _ptr(self.g_quat)
            g.opacity, g.sh = _ptr(self.g_opacity), _ptr(self.g_sh)
        else:
            K = SH_DIM[self.sh_degree]
            for k, rows in (("mean", 3), ("scale", 3), ("quat", 4), ("sh", 3 * K)):
                t = out[k]
                assert t.dtype == torch.float32 and t.is_contiguous() and tuple(t.shape) == (rows, self.n), k
            o = out["opacity"]
            assert o.dtype == torch.float32 and o.is_contiguous() and tuple(o.shape) == (self.n,)
            g.ld = max(self.n, 1)
            g.mean, g.scale, g.quat = _ptr(out["mean"]), _ptr(out["scale"]), _ptr(out["quat"])
            g.opacity, g.sh = _ptr(o), _ptr(out["sh"])
        g.grad2d = _ptr(self.grad2d)
        return g

    # -- stages -------------------------------------------------------------
    def project(self, g: DeviceGaussians, stream=None):
        assert g.n == self.n and g.sh_degree == self.sh_degree
        N.call("gs_project", C.byref(g.c_struct()), C.byref(self.c_cam), C.byref(self.c_opts),
               C.byref(self.c_proj()), C.c_void_p(stream_handle(stream)))

    def bin_sort(self, stream=None):
        N.call("gs_bin_sort", C.byref(self.c_proj()), self.n, C.byref(self.c_cam), C.byref(self.c_opts),
               C.byref(self.c_bins()), _ptr(self.ws), self.ws.numel(), C.c_void_p(stream_handle(stream)))

    def render_fwd(self, stream=None):
        N.call("gs_render_fwd", C.byref(self.c_proj()), C.byref(self.c_bins()), C.byref(self.c_cam),
               C.byref(self.c_opts), _ptr(self.image), _ptr(self.final_T), _ptr(self.n_contrib),
               C.c_void_p(stream_handle(stream)))

    def render_bwd(self, g: DeviceGaussians, dimg: torch.Tensor, stream=None, out: dict | None = None):
        assert self.has_grads, "frame was created without gradient buffers"
        assert dimg.shape == (3, self.H, self.W) and dimg.dtype == torch.float32 and dimg.is_contiguous()
        N.call("gs_render_bwd", C.byref(g.c_struct()), C.byref(self.c_cam), C.byref(self.c_opts),
               C.byref(self.c_proj()), C.byref(self.c_bins()), _ptr(self.final_T), _ptr(self.n_contrib),
               _ptr(dimg), C.byref(self.c_grads(out)), _ptr(self.bwd_ws), self.bwd_ws.numel() * 4,
               C.c_void_p(stream_handle(stream)))

    def stats(self, stream=None) -> dict:
        """Blend work counters of the current bins (synchronises)."""
        c = torch.zeros(4, dtype=torch.int64, device=self.device)
        N.call("gs_render_stats", C.byref(self.c_proj()), C.byref(self.c_bins()), C.byref(self.c_cam),
               C.byref(self.c_opts), _ptr(c), C.c_void_p(stream_handle(stream)))
        v = c.cpu().numpy()
        return dict(evaluated=int(v[0]), support=int(v[1]), blended=int(v[2]), evaluated_bwd=int(v[3]))

    # -- stored blend state (for comparison with the recomputing backward) --
    def state_bytes(self) -> int:
        nbytes = C.c_size_t(0)
        N.call("gs_render_state_bytes", C.byref(self.c_bins()), C.byref(self.c_opts), C.byref(nbytes))
        return int(nbytes.value)

    def render_fwd_stored(self, state: torch.Tensor, stream=None):
        N.call("gs_render_fwd_stored", C.byref(self.c_proj()), C.byref(self.c_bins()), C.byref(self.c_cam),
               C.byref(self.c_opts), _ptr(self.image), _ptr(self.final_T), _ptr(self.n_contrib), _ptr(state),
               state.numel() * state.element_size(), C.c_void_p(stream_handle(stream)))

    def render_bwd_stored(self, g: DeviceGaussians, dimg: torch.Tensor, state: torch.Tensor, stream=None,
                          out: dict | None = None):
        assert dimg.shape == (3, self.H, self.W) and dimg.dtype == torch.float32 and dimg.is_contiguous()
        N.call("gs_render_bwd_stored", C.byref(g.c_struct()), C.byref(self.c_cam), C.byref(self.c_opts),
               C.byref(self.c_proj()), C.byref(self.c_bins()), _ptr(self.final_T), _ptr(self.n_contrib),
               _ptr(state), state.numel() * state.element_size(), _ptr(dimg), C.byref(self.c_grads(out)),
               _ptr(self.bwd_ws), self.bwd_ws.numel() * 4, C.c_void_p(stream_handle(stream)))

    def forward(self, g: DeviceGaussians, stream=None):
        self.project(g, stream)
        self.bin_sort(stream)
        self.render_fwd(stream)

    # -- host checks (synchronise) -----------------------------------------
    def pairs(self) -> tuple[int, int]:
        pc = self.pair_count.cpu().numpy().astype(np.uint32)
        return int(pc[0]), int(pc[1])

    def check_status(self):
        st = int(self.status.item())
        if st != 0:
            raise N.GsError(st, f"device status (pairs needed {self.pairs()[1]}, capacity {self.capacity})")

    def ensure_capacity(self, g: DeviceGaussians, stream=None, headroom: float = 1.25) -> int:
        """Project and bin once; grow the pair buffers (and redo) when the
        view needs more pairs than the capacity.  Returns P."""
        self.project(g, stream)
        self.bin_sort(stream)
        if int(self.status.item()) == N.GS_ERR_CAPACITY:
            need = self.pairs()[1]
            self.set_capacity(int(math.ceil(need * headroom)) + 1024)
            self.bin_sort(stream)
            self.check_status()
        return self.pairs()[0]

    def grads(self) -> dict:
        n = self.n
        return dict(mean=self.g_mean[:, :n], scale=self.g_scale[:, :n], quat=self.g_quat[:, :n],
                    opacity=self.g_opacity[:n], sh=self.g_sh[:, :n], grad2d=self.grad2d[:, :n])


def render(g: DeviceGaussians, cam, tile=(16, 16), capacity=None) -> Frame:
    """Project, bin, sort and blend one view; returns the Frame holding the
    image, final transmittance, per-pixel contributor counts and the bins."""
    f = Frame(g.n, g.sh_degree, cam, tile, capacity)
    f.ensure_capacity(g)
    f.render_fwd()
    f.check_status()
    return f


def render_backward(f: Frame, g: DeviceGaussians, dimg: torch.Tensor) -> dict:
    f.render_bwd(g, dimg.contiguous())
    f.check_status()
    return f.grads()


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor, key_bits: int, count: int | None = None,
               stream=None) -> None:
    """In-place stable radix sort of int64 keys / int32 values on the device
    (the sort the binning runs)."""
    cap = keys.numel()
    assert vals.numel() == cap and keys.dtype == torch.int64 and vals.dtype == torch.int32
    cnt = torch.tensor([cap if count is None else count, 0], dtype=torch.int32, device=keys.device)
    nbytes = C.c_size_t(0)
    N.call("gs_sort_workspace", cap, key_bits, C.byref(nbytes))
    ws = torch.empty(max(int(nbytes.value), 1), dtype=torch.uint8, device=keys.device)
    N.call("gs_sort_pairs", _ptr(keys), _ptr(vals), _ptr(cnt), cap, key_bits, _ptr(ws), ws.numel(),
           C.c_void_p(stream_handle(stream)))
