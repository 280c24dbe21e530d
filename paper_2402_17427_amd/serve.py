"""Render server over a merged scene resident in HBM (gs_serve_* C ABI).

VastGaussian (arXiv 2402.17427), sections 4.3 and 5: the merged scene is
rendered from novel views in real time.  `Server` keeps the scene's device
planes alive, submits requests (camera + caller-owned output image) that the
native worker batches continuously, and waits for them with host-clock
timing statistics.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as N
from .raster import DeviceGaussians, _ptr


class gs_serve_config(C.Structure):
    _fields_ = [("memory_budget", C.c_int64), ("pipelines", C.c_int32), ("max_views", C.c_int32),
                ("max_queue", C.c_int32), ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("max_pixels", C.c_int64),
                ("widen_px", C.c_float), ("initial_pairs_per_slot", C.c_double), ("start_paused", C.c_int32),
                ("max_pairs", C.c_int64)]


class gs_request_stats(C.Structure):
    _fields_ = [("t_arrive_ns", C.c_int64), ("t_start_ns", C.c_int64), ("t_done_ns", C.c_int64),
                ("status", C.c_int32), ("batch_views", C.c_int32), ("attempts", C.c_int32), ("cells", C.c_int32),
                ("gaussians", C.c_int64)]


class gs_serve_stats(C.Structure):
    _fields_ = [("batches", C.c_int64), ("requeues", C.c_int64), ("max_batch_views", C.c_int64),
                ("queued", C.c_int64), ("pipelines", C.c_int32), ("slots_cap", C.c_int64), ("pairs_cap", C.c_int64),
                ("pixels_cap", C.c_int64), ("pairs_per_slot", C.c_double)]


N.register("gs_serve_create", [C.POINTER(N.gs_gaussians), C.c_void_p, C.c_void_p, C.c_int32,
                               C.POINTER(gs_serve_config), C.POINTER(C.c_void_p)])
N.register("gs_serve_submit", [C.c_void_p, C.POINTER(N.gs_camera), C.c_void_p, C.POINTER(C.c_uint64)])
N.register("gs_serve_wait", [C.c_void_p, C.c_uint64, C.c_int32, C.POINTER(gs_request_stats)])
N.register("gs_serve_info", [C.c_void_p, C.POINTER(gs_serve_stats)])
N.register("gs_serve_resume", [C.c_void_p])
N.register("gs_serve_destroy", [C.c_void_p], None)


class Server:
    def __init__(self, scene: DeviceGaussians, cell_aabbs, cell_offsets, memory_budget=8 << 30, pipelines=2,
                 max_views=8, max_queue=1024, tile=(16, 16), max_pixels=4 * 3840 * 2160, widen_px=64.0,
                 initial_pairs_per_slot=3.0, start_paused=False, max_pairs=0):
        self.scene = scene
        self.boxes = np.ascontiguousarray(cell_aabbs, np.float32)
        self.offsets = np.ascontiguousarray(cell_offsets, np.int64)
        n_cells = self.boxes.shape[0]
        assert self.boxes.shape == (n_cells, 6) and self.offsets.shape == (n_cells + 1,)
        cfg = gs_serve_config(int(memory_budget), int(pipelines), int(max_views), int(max_queue), int(tile[0]),
                              int(tile[1]), int(max_pixels), float(widen_px), float(initial_pairs_per_slot),
                              int(bool(start_paused)), int(max_pairs))
        self._c_scene = scene.c_struct()
        h = C.c_void_p(0)
        N.call("gs_serve_create", C.byref(self._c_scene), self.boxes.ctypes.data_as(C.c_void_p),
               self.offsets.ctypes.data_as(C.c_void_p), n_cells, C.byref(cfg), C.byref(h))
        self._h = h
        self._outs = {}

    def submit(self, cam, out: torch.Tensor) -> int:
        """Queue a render of `cam` into `out` ([3][H][W] float32 CUDA,
        untouched until wait() returns for the ticket)."""
        assert out.dtype == torch.float32 and out.is_contiguous() and out.is_cuda
        assert tuple(out.shape) == (3, int(cam.height), int(cam.width))
        # the server renders on its own streams: whatever torch queued on
        # `out` must be finished first
        torch.cuda.current_stream(out.device).synchronize()
        t = C.c_uint64(0)
        c = N.make_camera(cam)
        N.call("gs_serve_submit", self._h, C.byref(c), _ptr(out), C.byref(t))
        self._outs[int(t.value)] = out
        return int(t.value)

    def wait(self, ticket: int, timeout_ms: int = -1) -> dict:
        st = gs_request_stats()
        try:
            N.call("gs_serve_wait", self._h, ticket, int(timeout_ms), C.byref(st))
        finally:
            if st.t_done_ns or st.status:
                self._outs.pop(ticket, None)
        return dict(t_arrive_ns=st.t_arrive_ns, t_start_ns=st.t_start_ns, t_done_ns=st.t_done_ns,
                    status=st.status, batch_views=st.batch_views, attempts=st.attempts, cells=st.cells,
                    gaussians=st.gaussians, latency_ms=(st.t_done_ns - st.t_arrive_ns) * 1e-6)

    def resume(self):
        N.call("gs_serve_resume", self._h)

    def info(self) -> dict:
        s = gs_serve_stats()
        N.call("gs_serve_info", self._h, C.byref(s))
        return {k: getattr(s, k) for k, _ in gs_serve_stats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            N.lib().gs_serve_destroy(self._h)
            self._h = C.c_void_p(0)
            self._outs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
