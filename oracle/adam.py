"""FP64 CPU oracle for the optimiser step -- TEST INFRASTRUCTURE.

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's `cpu_baseline`
leg may import this module; the GPU optimiser kernel shares nothing with it.

What it computes (VastGaussian, arXiv 2402.17427, section 3): the Gaussians'
properties are optimised by gradient descent on the loss of Eq. 1, and the
optimisation is interleaved with adaptive densification, triggered by each
point's cumulative gradient; every setting the paper does not list is that
of 3DGS (section 5.1).  The readings taken from 3DGS:
  * the optimised (raw) properties are the position, log-scale (scale =
    exp), the un-normalised quaternion, the opacity logit (opacity =
    sigmoid) and the SH coefficients; the renderer's gradient, taken w.r.t.
    the activated values, reaches the raw ones by the chain rule
    (d/d log s = s d/ds, d/d logit o = o (1 - o) d/do);
  * the optimiser is Adam (Kingma and Ba) with bias correction, one
    learning rate per property group (position, scale, rotation, opacity,
    SH DC, SH rest), every Gaussian updated every step (a zero gradient
    still moves a parameter through its first moment);
  * densification statistics: for every Gaussian visible in the step's
    view (non-empty tile rectangle) the norm of its image-space centre
    gradient (dL/du, dL/dv, in pixels) is added to an accumulator and a
    visibility count is incremented; the densify/prune policy that reads
    them is not part of the step.
Planes follow the order mean 3, log-scale 3, quaternion 4, opacity logit 1,
SH 3K (plane c*K + j), each [n] float64.
"""
from __future__ import annotations

import numpy as np


def plane_groups(sh_degree: int):
    """(name, first plane, count) of each learning-rate group."""
    K = (sh_degree + 1) ** 2
    groups = [("mean", 0, 3), ("scale", 3, 3), ("quat", 6, 4), ("opacity", 10, 1)]
    return groups, K


def lr_of_planes(cfg: dict, sh_degree: int) -> np.ndarray:
    """Learning rate of every plane: SH plane c*K + j takes lr_sh_dc for
    j = 0 and lr_sh_rest otherwise."""
    groups, K = plane_groups(sh_degree)
    lr = np.zeros(11 + 3 * K)
    for name, p0, cnt in groups:
        lr[p0:p0 + cnt] = cfg["lr_" + name]
    for c in range(3):
        for j in range(K):
            lr[11 + c * K + j] = cfg["lr_sh_dc"] if j == 0 else cfg["lr_sh_rest"]
    return lr


def activated(raw: np.ndarray) -> dict:
    """Scale and opacity the renderer sees for raw planes [11 + 3K][n]."""
    raw = np.asarray(raw, np.float64)
    return dict(scale=np.exp(raw[3:6]), opacity=1.0 / (1.0 + np.exp(-raw[10])))


def raw_gradient(raw, grad_act) -> np.ndarray:
    """Chain rule from the renderer's gradient (planes in the same order,
    w.r.t. the activated scale and opacity) to the raw planes."""
    raw = np.asarray(raw, np.float64)
    g = np.array(grad_act, np.float64, copy=True)
    act = activated(raw)
    g[3:6] *= act["scale"]
    o = act["opacity"]
    g[10] *= o * (1.0 - o)
    return g


def adam_step(raw, m, v, grad_act, cfg: dict, sh_degree: int, step: int):
    """One Adam step (t = step, 1-based) on every plane.  Returns (raw, m, v)."""
    raw = np.asarray(raw, np.float64)
    g = raw_gradient(raw, grad_act)
    b1, b2, eps = cfg["beta1"], cfg["beta2"], cfg["eps"]
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    m_hat = m / (1.0 - b1 ** step)
    v_hat = v / (1.0 - b2 ** step)
    lr = lr_of_planes(cfg, sh_degree)[:, None]
    return raw - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def densify_stats(accum, count, grad_uv, visible):
    """accum += |(dL/du, dL/dv)| and count += 1 where visible."""
    accum = np.array(accum, np.float64, copy=True)
    count = np.array(count, np.float64, copy=True)
    gu, gv = np.asarray(grad_uv[0], np.float64), np.asarray(grad_uv[1], np.float64)
    vis = np.asarray(visible, bool)
    accum[vis] += np.sqrt(gu[vis] ** 2 + gv[vis] ** 2)
    count[vis] += 1.0
    return accum, count


# 3DGS defaults (position rate before its decay schedule, for a unit extent)
DEFAULTS = dict(lr_mean=1.6e-4, lr_scale=5e-3, lr_quat=1e-3, lr_opacity=5e-2, lr_sh_dc=2.5e-3,
                lr_sh_rest=2.5e-3 / 20.0, beta1=0.9, beta2=0.999, eps=1e-15)
