"""Torch-facing wrapper of the fused training loss (gs_loss in gs.h).

Eq. 1 of VastGaussian (arXiv 2402.17427, section 3): (1 - lambda) L1 +
lambda D-SSIM between a rendered image and its ground truth, or Eq. 3
(section 4.2) with the L1 term on the appearance-adjusted image.  The
value and the image gradients come from the HIP kernels behind libgsmi.so;
this module only sizes buffers and passes pointers and the stream.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _native as N
from .raster import _ptr, stream_handle

LAMBDA = 0.2


def workspace_bytes(channels: int, width: int, height: int) -> int:
    b = C.c_size_t()
    N.call("gs_loss_workspace", channels, width, height, C.byref(b))
    return int(b.value)


class ImageLoss:
    """Buffers for the loss of one image shape ([C][H][W] float32 cuda),
    so that a timed loop allocates nothing."""

    def __init__(self, channels: int, height: int, width: int, device="cuda", appearance: bool = False):
        self.shape = (channels, height, width)
        self.loss = torch.zeros(3, dtype=torch.float32, device=device)
        self.d_image = torch.empty(self.shape, dtype=torch.float32, device=device)
        self.d_image_l1 = torch.empty(self.shape, dtype=torch.float32, device=device) if appearance else None
        nb = workspace_bytes(channels, width, height)
        self.ws = torch.empty((nb + 7) // 8, dtype=torch.float64, device=device)
        self.ws_bytes = nb

    def _check(self, name, t):
        if t.dtype != torch.float32 or not t.is_cuda or tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name}: expected contiguous float32 cuda {list(self.shape)}, got "
                             f"{t.dtype} {tuple(t.shape)}")

    def __call__(self, image, target, lam: float = LAMBDA, image_l1=None, stream=None):
        """Enqueue the loss; returns (loss[3] = total, L1, mean SSIM;
        d_image; d_image_l1 or None).  The returned tensors are this
        object's buffers, overwritten by the next call."""
        self._check("image", image)
        self._check("target", target)
        if image_l1 is not None:
            self._check("image_l1", image_l1)
            if self.d_image_l1 is None:
                self.d_image_l1 = torch.empty(self.shape, dtype=torch.float32, device=image.device)
        c, h, w = self.shape
        N.call("gs_loss", _ptr(image), _ptr(image_l1), _ptr(target), c, w, h, float(lam), _ptr(self.loss),
               _ptr(self.d_image), _ptr(self.d_image_l1) if image_l1 is not None else None, _ptr(self.ws),
               self.ws_bytes, C.c_void_p(stream_handle(stream)))
        return self.loss, self.d_image, (self.d_image_l1 if image_l1 is not None else None)


def image_loss(image, target, lam: float = LAMBDA, image_l1=None, stream=None):
    """One-shot form of ImageLoss: (loss[3], d_image, d_image_l1 or None)."""
    c, h, w = image.shape
    return ImageLoss(c, h, w, device=image.device, appearance=image_l1 is not None)(image, target, lam, image_l1,
                                                                                     stream)
