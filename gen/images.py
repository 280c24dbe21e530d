"""Seeded synthetic image pairs for the training loss.

This module only draws inputs: a ground-truth image and a rendered image of
the same view, planar [C][H][W] float32.  It holds none of the loss
arithmetic (no window, no statistics), so the FP64 oracle and the HIP path
can both consume its outputs.

The pairs stand in for the aerial training photographs and the renders of a
partly optimised cell (VastGaussian, arXiv 2402.17427, sections 4.2 and
5.1), which are not available: the target is a city-like image (smooth
shading, axis-aligned blocks with sharp edges, fine texture) in [0, 1]; the
render is that image slightly blurred and shifted in colour, with its own
noise and a few blotches, so that both the SSIM and the L1 terms are far
from their optimum and the render can exceed 1 as an unclamped render can.
"""
from __future__ import annotations

import numpy as np


def _smooth(rng, C, H, W, cells):
    """Bilinear upsample of a coarse random grid: low-frequency shading."""
    gy, gx = max(2, H // cells + 2), max(2, W // cells + 2)
    coarse = rng.uniform(0.0, 1.0, (C, gy, gx))
    ys = np.linspace(0.0, gy - 1.001, H)
    xs = np.linspace(0.0, gx - 1.001, W)
    y0 = ys.astype(np.int64)
    x0 = xs.astype(np.int64)
    fy = (ys - y0)[None, :, None]
    fx = (xs - x0)[None, None, :]
    a = coarse[:, y0][:, :, x0]
    b = coarse[:, y0][:, :, x0 + 1]
    c = coarse[:, y0 + 1][:, :, x0]
    d = coarse[:, y0 + 1][:, :, x0 + 1]
    return (1 - fy) * ((1 - fx) * a + fx * b) + fy * ((1 - fx) * c + fx * d)


def image_pair(seed, width, height, channels=3, n_blocks=None):
    """(rendered, target), each float32 [channels][height][width]."""
    rng = np.random.default_rng(seed)
    C, H, W = channels, height, width
    t = 0.6 * _smooth(rng, C, H, W, 64)
    nb = n_blocks if n_blocks is not None else max(4, (H * W) // 4000)
    for _ in range(nb):
        h = int(rng.integers(2, max(3, H // 6)))
        w = int(rng.integers(2, max(3, W // 6)))
        y = int(rng.integers(0, H))
        x = int(rng.integers(0, W))
        t[:, y:y + h, x:x + w] = rng.uniform(0.0, 1.0, (C, 1, 1))
    t += 0.04 * rng.standard_normal((C, H, W))
    t = np.clip(t, 0.0, 1.0)
    # render: 3-tap blur of the target, a colour shift, noise and blotches
    r = t.copy()
    r[:, 1:-1, :] = 0.25 * t[:, :-2, :] + 0.5 * t[:, 1:-1, :] + 0.25 * t[:, 2:, :]
    r2 = r.copy()
    r2[:, :, 1:-1] = 0.25 * r[:, :, :-2] + 0.5 * r[:, :, 1:-1] + 0.25 * r[:, :, 2:]
    r = r2 * rng.uniform(0.9, 1.1, (C, 1, 1)) + rng.uniform(-0.03, 0.03, (C, 1, 1))
    r += 0.02 * rng.standard_normal((C, H, W))
    for _ in range(max(1, nb // 4)):
        h = int(rng.integers(2, max(3, H // 10)))
        w = int(rng.integers(2, max(3, W // 10)))
        y = int(rng.integers(0, H))
        x = int(rng.integers(0, W))
        r[:, y:y + h, x:x + w] += rng.uniform(-0.3, 0.3, (C, 1, 1))
    r = np.maximum(r, 0.0)
    return np.ascontiguousarray(r, np.float32), np.ascontiguousarray(t, np.float32)
