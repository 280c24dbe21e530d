"""Progressive data partitioning (gs_partition_views / gs_select_points /
gs_merge_keep in gs.h).

VastGaussian (arXiv 2402.17427), section 4.1: region division by camera
positions, 20 % boundary expansion, airspace-aware visibility-based camera
selection and coverage-based point selection; section 4.3: each cell keeps
the Gaussians inside its original rectangle.  The view side runs on the
host in the C++ library, the point selection and the merge mask in HIP
kernels; this module only marshals arrays.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as N
from .raster import _ptr, stream_handle

EXPAND = 0.2
VISIBILITY = 0.25


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def partition_views(cams, points_host, m: int, n: int, expand: float = EXPAND,
                    threshold: float = VISIBILITY) -> dict:
    """Host step: dict bounds, expanded [m n][4], boxes [m n][6],
    visibility, view_member [m n][V] (0 / 1 position / 2 visibility)."""
    V = len(cams)
    c_cams = (N.gs_camera * V)(*[N.make_camera(c) for c in cams])
    pts = np.ascontiguousarray(points_host, np.float32).reshape(-1, 3)
    cfg = N.gs_partition_config(int(m), int(n), float(expand), float(threshold))
    nc = m * n
    out = dict(bounds=np.zeros((nc, 4)), expanded=np.zeros((nc, 4)), boxes=np.zeros((nc, 6)),
               visibility=np.zeros((nc, V)), view_member=np.zeros((nc, V), np.uint8))
    N.call("gs_partition_views", c_cams, V, _np_ptr(pts), pts.shape[0], C.byref(cfg), _np_ptr(out["bounds"]),
           _np_ptr(out["expanded"]), _np_ptr(out["boxes"]), _np_ptr(out["visibility"]), _np_ptr(out["view_member"]))
    return out


class PointSelector:
    """Device buffers of the point selection for fixed view and cell counts."""

    def __init__(self, n_views: int, n_cells: int, n_points: int, device="cuda"):
        b = C.c_size_t()
        N.call("gs_select_points_workspace", n_views, n_cells, n_points, C.byref(b))
        self.n_points = n_points
        self.ws = torch.empty((int(b.value) + 7) // 8, dtype=torch.float64, device=device)
        self.ws_bytes = int(b.value)
        self.n_views, self.n_cells = n_views, n_cells

    def __call__(self, points_dev: torch.Tensor, cams, expanded, view_member, tests=None, out=None, stream=None):
        """points_dev: [3][N] float32 cuda.  Returns uint8 [n_cells][N] (0 /
        1 position / 2 coverage)."""
        assert points_dev.dtype == torch.float32 and points_dev.dim() == 2 and points_dev.shape[0] == 3
        npts = points_dev.shape[1]
        assert npts <= self.n_points, "workspace sized for fewer points"
        ld = points_dev.stride(0)
        c_cams = (N.gs_camera * len(cams))(*[N.make_camera(c) for c in cams])
        ex = np.ascontiguousarray(expanded, np.float64)
        vm = np.ascontiguousarray(view_member, np.uint8)
        if out is None:
            out = torch.empty((self.n_cells, max(npts, 1)), dtype=torch.uint8, device=points_dev.device)
        N.call("gs_select_points", _ptr(points_dev), npts, ld, c_cams, len(cams), _np_ptr(ex), self.n_cells,
               _np_ptr(vm), _ptr(out), _ptr(tests) if tests is not None else None, _ptr(self.ws), self.ws_bytes,
               C.c_void_p(stream_handle(stream)))
        return out


def merge_keep(mean: torch.Tensor, rect, closed=(False, False), stream=None) -> torch.Tensor:
    """uint8 [N]: 1 for the Gaussians whose (x, z) lies in the rectangle."""
    n = mean.shape[1]
    keep = torch.empty(max(n, 1), dtype=torch.uint8, device=mean.device)
    r = np.ascontiguousarray(rect, np.float64)
    N.call("gs_merge_keep", _ptr(mean), n, mean.stride(0), _np_ptr(r), int(bool(closed[0])), int(bool(closed[1])),
           _ptr(keep), C.c_void_p(stream_handle(stream)))
    return keep[:n]
