"""Torch-facing wrapper of the optimiser step (gs_adam_step in gs.h).

Section 3 of VastGaussian (arXiv 2402.17427): the Gaussians are optimised
by gradient descent on the loss, interleaved with densification driven by
each point's cumulative gradient; section 5.1 leaves the optimiser to
3DGS (Adam over the raw properties).  The update itself runs in the HIP
kernel behind libgsmi.so; this module holds the buffers and the step
count, and converts the initial activated values to raw ones once, on the
host.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _native as N
from .raster import SH_DIM, DeviceGaussians, Frame, _ptr, stream_handle

# 3DGS defaults; the position rate is for a unit scene extent and is decayed
# by the caller's schedule
DEFAULTS = dict(lr_mean=1.6e-4, lr_scale=5e-3, lr_quat=1e-3, lr_opacity=5e-2, lr_sh_dc=2.5e-3,
                lr_sh_rest=2.5e-3 / 20.0, beta1=0.9, beta2=0.999, eps=1e-15)


def config(step: int, **kw) -> N.gs_adam_config:
    c = N.gs_adam_config()
    d = dict(DEFAULTS, **kw)
    for k in ("lr_mean", "lr_scale", "lr_quat", "lr_opacity", "lr_sh_dc", "lr_sh_rest", "beta1", "beta2", "eps"):
        setattr(c, k, float(d[k]))
    c.step = int(step)
    return c


class Adam:
    """Optimiser of one Gaussian set.  `dg` is the set the rasterizer reads:
    its mean, quat and sh planes are the raw properties (updated in place),
    its scale and opacity planes are rewritten from the raw log-scale and
    opacity logit kept here.  Moments start at zero; the densification
    statistics (grad_accum, visible_count) accumulate over steps."""

    def __init__(self, dg: DeviceGaussians, log_scale: torch.Tensor, logit_opacity: torch.Tensor,
                 stats: bool = True, **hyper):
        self.dg = dg
        self.log_scale = log_scale
        self.logit_opacity = logit_opacity
        n, K = dg.n, SH_DIM[dg.sh_degree]
        planes = 11 + 3 * K
        dev = dg.mean.device
        self.m = torch.zeros((planes, max(n, 1)), dtype=torch.float32, device=dev)
        self.v = torch.zeros_like(self.m)
        self.grad_accum = torch.zeros(max(n, 1), dtype=torch.float32, device=dev) if stats else None
        self.visible_count = torch.zeros_like(self.grad_accum) if stats else None
        self.hyper = hyper
        self.t = 0

    @classmethod
    def from_activated(cls, dg: DeviceGaussians, **kw) -> "Adam":
        """Raw log-scale and logit from the set's activated values (host,
        once); the activated planes are then rewritten from them on the
        device by the first step."""
        s = dg.scale.detach().cpu().numpy().astype(np.float64)
        o = np.clip(dg.opacity.detach().cpu().numpy().astype(np.float64), 1e-7, 1 - 1e-7)
        ls = torch.as_tensor(np.log(s).astype(np.float32)).to(dg.mean.device)
        lo = torch.as_tensor(np.log(o / (1.0 - o)).astype(np.float32)).to(dg.mean.device)
        return cls(dg, ls, lo, **kw)

    def c_params(self) -> N.gs_params:
        p = N.gs_params()
        p.n = self.dg.n
        p.ld = self.dg.ld
        p.sh_degree = self.dg.sh_degree
        p.mean, p.log_scale, p.quat = _ptr(self.dg.mean), _ptr(self.log_scale), _ptr(self.dg.quat)
        p.logit_opacity, p.sh = _ptr(self.logit_opacity), _ptr(self.dg.sh)
        return p

    def c_state(self) -> N.gs_adam_state:
        s = N.gs_adam_state()
        s.m, s.v = _ptr(self.m), _ptr(self.v)
        s.grad_accum, s.visible_count = _ptr(self.grad_accum), _ptr(self.visible_count)
        return s

    def step_grads(self, grads: N.gs_grads, tiles_touched=None, status=None, stream=None, **override):
        """One step from a gs_grads struct (device gradient planes)."""
        self.t += 1
        cfg = config(self.t, **dict(self.hyper, **override))
        use_stats = tiles_touched is not None and self.grad_accum is not None
        N.call("gs_adam_step", C.byref(self.c_params()), _ptr(self.dg.scale), _ptr(self.dg.opacity),
               C.byref(self.c_state()), C.byref(grads), _ptr(tiles_touched) if use_stats else None,
               _ptr(status) if status is not None else None, C.byref(cfg), C.c_void_p(stream_handle(stream)))

    def step(self, frame: Frame, stream=None, **override):
        """One step with the gradients and visibility the frame's last
        backward left (skipped on the device when its status is set)."""
        self.step_grads(frame.c_grads(), frame.tiles_touched, frame.status, stream, **override)
