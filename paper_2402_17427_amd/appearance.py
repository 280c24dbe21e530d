"""Torch-facing wrapper of the decoupled appearance model
(gs_appearance_* in gs.h).

VastGaussian (arXiv 2402.17427), section 4.2 and supplement S1.1: a CNN
on the 32x downsampled render concatenated with a per-image appearance
embedding yields a transformation map M, and the L1 term of Eq. 3 is taken
on I^a = I^r * M.  Every layer runs in the HIP kernels behind libgsmi.so;
this module holds the buffers (parameters, workspace) and passes pointers.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as N
from .raster import _ptr, stream_handle

EMBED = 64


def param_count(embed_dim: int = EMBED) -> int:
    n = C.c_int64()
    N.call("gs_appearance_param_count", embed_dim, C.byref(n))
    return int(n.value)


def layer_shapes(embed_dim: int = EMBED):
    return [(256, 3 + embed_dim), (128, 64), (64, 32), (32, 16), (16, 8), (16, 16), (3, 16)]


def pack(layers) -> np.ndarray:
    """Flatten [(weight [Cout][Cin][3][3], bias [Cout])] in layer order."""
    return np.concatenate([np.concatenate([np.ravel(w), np.ravel(b)]) for w, b in layers]).astype(np.float32)


def unpack(flat, embed_dim: int = EMBED):
    out, o = [], 0
    for co, ci in layer_shapes(embed_dim):
        n = co * ci * 9
        out.append((flat[o:o + n].reshape(co, ci, 3, 3), flat[o + n:o + n + co]))
        o += n + co
    return out


class AppearanceModel:
    """Buffers of the appearance model for one image size."""

    def __init__(self, height: int, width: int, params: torch.Tensor, embed_dim: int = EMBED, device="cuda"):
        self.H, self.W, self.m = int(height), int(width), int(embed_dim)
        assert params.dtype == torch.float32 and params.is_cuda and params.numel() == param_count(self.m)
        self.params = params
        b = C.c_size_t()
        N.call("gs_appearance_workspace", self.W, self.H, self.m, C.byref(b))
        self.ws = torch.empty((int(b.value) + 255) // 4, dtype=torch.float32, device=device)
        off = (-self.ws.data_ptr()) % 256      # 256-byte aligned view
        self.ws_ptr = C.c_void_p(self.ws.data_ptr() + off)
        self.ws_bytes = self.ws.numel() * 4 - off
        self.image_adj = torch.empty((3, self.H, self.W), dtype=torch.float32, device=device)
        self.transform = torch.empty_like(self.image_adj)
        self.d_params = torch.empty_like(params)
        self.d_embedding = torch.empty(max(self.m, 1), dtype=torch.float32, device=device)

    def forward(self, image: torch.Tensor, embedding: torch.Tensor, stream=None):
        """I^a (and M in self.transform)."""
        N.call("gs_appearance_fwd", _ptr(image), self.W, self.H, _ptr(embedding), self.m, _ptr(self.params),
               _ptr(self.image_adj), _ptr(self.transform), self.ws_ptr, self.ws_bytes,
               C.c_void_p(stream_handle(stream)))
        return self.image_adj

    def backward(self, image, embedding, d_image_adj, d_image, stream=None):
        """Adds dL/dI^r into d_image; returns (d_embedding, d_params)."""
        N.call("gs_appearance_bwd", _ptr(image), self.W, self.H, _ptr(embedding), self.m, _ptr(self.params),
               _ptr(d_image_adj), _ptr(d_image), _ptr(self.d_embedding), _ptr(self.d_params), self.ws_ptr,
               self.ws_bytes, C.c_void_p(stream_handle(stream)))
        return self.d_embedding[:self.m], self.d_params
