"""Batched training step over several partition cells (gs_batch_* C ABI).

VastGaussian (arXiv 2402.17427), section 4.1: the scene's cells are
optimised independently.  `BatchStep` runs one training step (render, loss,
backward, and optionally the optimiser step) of several cells of uneven
sizes at once, each stage one launch over all cells, captured as a hipGraph
and replayed per `step()`.  The loss is L1, or Eq. 1 (L1 + D-SSIM) with
`loss_lambda` > 0; with `optimizers` (one optim.Adam per cell, built on the
same DeviceGaussians) every replay ends with each cell's Adam step and
densification statistics.  Outputs live in torch tensors owned by this
object (the graph writes into them): `image(c)`, `grads[c]`, `loss`.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _native as N
from .raster import SH_DIM, DeviceGaussians, _ptr, stream_handle


class gs_batch_optim(C.Structure):
    _fields_ = [("params", C.POINTER(N.gs_params)), ("states", C.POINTER(N.gs_adam_state)),
                ("hyper", N.gs_adam_config), ("lr_mean_final", C.c_float), ("lr_mean_steps", C.c_int32)]


class gs_batch_config(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("persistent", C.c_int32), ("use_graph", C.c_int32),
                ("autotune", C.c_int32), ("capacity_headroom", C.c_double), ("loss_lambda", C.c_float),
                ("optim", C.POINTER(gs_batch_optim)), ("fwd_batch", C.c_int32), ("item_cap", C.c_int32),
                ("grid_pct", C.c_int32)]


class gs_batch_stats(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("persistent", C.c_int32), ("use_graph", C.c_int32),
                ("grid_fwd", C.c_int32), ("grid_bwd", C.c_int32), ("n_tiles", C.c_uint32), ("slots", C.c_int64),
                ("pair_capacity", C.c_int64), ("n_candidates", C.c_int32), ("cand_tile_w", C.c_int32 * 16),
                ("cand_tile_h", C.c_int32 * 16), ("cand_persistent", C.c_int32 * 16), ("cand_ms", C.c_double * 16),
                ("fwd_batch", C.c_int32), ("item_cap", C.c_int32), ("grid_pct", C.c_int32),
                ("cand_fwd_batch", C.c_int32 * 16), ("cand_item_cap", C.c_int32 * 16),
                ("cand_grid_pct", C.c_int32 * 16)]


N.register("gs_batch_create", [C.POINTER(N.gs_gaussians), C.POINTER(N.gs_camera), C.POINTER(C.c_void_p), C.c_int32,
                               C.c_void_p, C.POINTER(N.gs_grads), C.c_void_p, C.POINTER(gs_batch_config),
                               C.c_void_p, C.POINTER(C.c_void_p)])
N.register("gs_batch_step", [C.c_void_p, C.c_void_p])
N.register("gs_batch_info", [C.c_void_p, C.POINTER(gs_batch_stats)])
N.register("gs_batch_status", [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_uint32)])
N.register("gs_batch_destroy", [C.c_void_p], None)


class BatchStep:
    def __init__(self, cells: list[DeviceGaussians], cams, targets: list[torch.Tensor], tile=(16, 16),
                 persistent=True, use_graph=True, autotune=False, headroom=1.25, stream=None,
                 loss_lambda: float = 0.0, optimizers=None, lr_mean_final: float = 0.0, lr_mean_steps: int = 0,
                 fwd_batch: int = 0, item_cap: int = 0, grid_pct: int = 0, **hyper):
        n = len(cells)
        assert n == len(cams) == len(targets) and n > 0
        dev = cells[0].mean.device
        self.cells, self.cams = cells, cams
        self.targets = [t.contiguous().float() for t in targets]
        self.sizes = [(int(c.height), int(c.width)) for c in cams]
        offs, o = [], 0
        for (h, w) in self.sizes:
            offs.append(o)
            o += 3 * h * w
        self.img_offsets = offs
        self.images = torch.zeros(max(o, 1), dtype=torch.float32, device=dev)
        self.loss = torch.zeros(n, dtype=torch.float32, device=dev)
        self.grads = []
        c_grads = (N.gs_grads * n)()
        for i, g in enumerate(cells):
            K = SH_DIM[g.sh_degree]
            m = max(g.n, 1)
            gr = dict(mean=torch.zeros((3, m), device=dev), scale=torch.zeros((3, m), device=dev),
                      quat=torch.zeros((4, m), device=dev), opacity=torch.zeros(m, device=dev),
                      sh=torch.zeros((3 * K, m), device=dev))
            self.grads.append(gr)
            c_grads[i].ld = m
            c_grads[i].mean, c_grads[i].scale, c_grads[i].quat = _ptr(gr["mean"]), _ptr(gr["scale"]), _ptr(gr["quat"])
            c_grads[i].opacity, c_grads[i].sh = _ptr(gr["opacity"]), _ptr(gr["sh"])
            c_grads[i].grad2d = C.c_void_p(0)
        for i, (t, (h, w)) in enumerate(zip(self.targets, self.sizes)):
            assert tuple(t.shape) == (3, h, w), (i, t.shape)
        c_cells = (N.gs_gaussians * n)(*[g.c_struct() for g in cells])
        c_cams = (N.gs_camera * n)(*[N.make_camera(c) for c in cams])
        c_tg = (C.c_void_p * n)(*[t.data_ptr() for t in self.targets])
        cfg = gs_batch_config(int(tile[0]), int(tile[1]), int(bool(persistent)), int(bool(use_graph)),
                              int(bool(autotune)), float(headroom), float(loss_lambda), None, int(fwd_batch),
                              int(item_cap), int(grid_pct))
        keep_opt = None
        if optimizers is not None:
            from . import optim
            assert len(optimizers) == n
            for o, g in zip(optimizers, cells):
                assert o.dg is g, "each optimizer must hold its cell's DeviceGaussians"
                assert o.grad_accum is not None, "the batch keeps the densification statistics"
            c_par = (N.gs_params * n)(*[o.c_params() for o in optimizers])
            c_st = (N.gs_adam_state * n)(*[o.c_state() for o in optimizers])
            first = optimizers[0].t + 1
            opt = gs_batch_optim(c_par, c_st, optim.config(first, **hyper), float(lr_mean_final), int(lr_mean_steps))
            cfg.optim = C.pointer(opt)
            keep_opt = (c_par, c_st, opt)
        h = C.c_void_p(0)
        N.call("gs_batch_create", c_cells, c_cams, c_tg, n, _ptr(self.images), c_grads, _ptr(self.loss),
               C.byref(cfg), C.c_void_p(stream_handle(stream)), C.byref(h))
        self._h = h
        self._keep = (c_cells, c_cams, c_tg, c_grads, keep_opt)

    def step(self, stream=None):
        N.call("gs_batch_step", self._h, C.c_void_p(stream_handle(stream)))

    def image(self, c: int) -> torch.Tensor:
        h, w = self.sizes[c]
        o = self.img_offsets[c]
        return self.images[o:o + 3 * h * w].view(3, h, w)

    def cell_grads(self, c: int) -> dict:
        n = self.cells[c].n
        return {k: (v[..., :n] if v.dim() == 2 else v[:n]) for k, v in self.grads[c].items()}

    def info(self) -> dict:
        s = gs_batch_stats()
        N.call("gs_batch_info", self._h, C.byref(s))
        cands = [dict(tile=(s.cand_tile_w[i], s.cand_tile_h[i]), persistent=bool(s.cand_persistent[i]),
                      fwd_batch=s.cand_fwd_batch[i], item_cap=s.cand_item_cap[i], grid_pct=s.cand_grid_pct[i],
                      ms=s.cand_ms[i]) for i in range(s.n_candidates)]
        return dict(tile=(s.tile_w, s.tile_h), persistent=bool(s.persistent), use_graph=bool(s.use_graph),
                    grid_fwd=s.grid_fwd, grid_bwd=s.grid_bwd, fwd_batch=s.fwd_batch, item_cap=s.item_cap,
                    grid_pct=s.grid_pct, n_tiles=s.n_tiles, slots=s.slots, pair_capacity=s.pair_capacity,
                    candidates=cands)

    def status(self, stream=None):
        st = C.c_int32(0)
        pairs = (C.c_uint32 * 2)()
        N.call("gs_batch_status", self._h, C.c_void_p(stream_handle(stream)), C.byref(st), pairs)
        return int(st.value), (int(pairs[0]), int(pairs[1]))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            N.lib().gs_batch_destroy(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
