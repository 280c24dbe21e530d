"""FP64 CPU oracle for the training loss -- TEST INFRASTRUCTURE.

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's `cpu_baseline`
leg may import this module; the GPU loss kernel shares nothing with it.

What it computes (VastGaussian, arXiv 2402.17427): the per-image loss of
Eq. 1 (section 3), a (1 - lambda) weighted L1 term plus a lambda weighted
D-SSIM term between the rendered image and its ground truth, and its
Eq. 3 form (section 4.2), where the L1 term is taken on the
appearance-adjusted image I^a while D-SSIM stays on the rendered image I^r.
The paper takes D-SSIM from 3DGS and fixes no constants; the readings used
here (the 3DGS ones) are:
  * D-SSIM = 1 - SSIM, SSIM averaged over every pixel and channel;
  * SSIM of Wang et al. with an 11 x 11 Gaussian window of sigma 1.5
    (normalised to sum 1), C1 = 0.01^2 and C2 = 0.03^2 (dynamic range 1);
  * the window statistics are zero-padded window sums at the borders:
    mu = sum w x, sigma^2 = sum w x^2 - mu^2, sigma_xy = sum w x y - mu_x mu_y,
    with x = y = 0 outside the image;
  * L1 = mean |I - I*| over every pixel and channel; its gradient uses
    sign(0) = 0; lambda = 0.2 by default.
Images are [C][H][W] arrays.  Everything is float64.  The statistics are
computed as plain window sums over the 121 offsets (no separable
filtering), and the gradient is the chain rule through those sums.
"""
from __future__ import annotations

import numpy as np

WINDOW = 11
SIGMA = 1.5
C1 = 0.01 ** 2
C2 = 0.03 ** 2
LAMBDA = 0.2


def window_1d(size: int = WINDOW, sigma: float = SIGMA) -> np.ndarray:
    """Sampled Gaussian exp(-k^2 / (2 sigma^2)), k = -(size//2)..size//2,
    normalised to sum 1."""
    k = np.arange(size, dtype=np.float64) - size // 2
    g = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return g / g.sum()


def window_2d() -> np.ndarray:
    g = window_1d()
    return np.outer(g, g)


def _window_sum(a: np.ndarray, w2: np.ndarray) -> np.ndarray:
    """out[c, i, j] = sum_{di, dj} w2[di, dj] * a[c, i + di - r, j + dj - r],
    with a = 0 outside the image (r = half window)."""
    C, H, W = a.shape
    r = w2.shape[0] // 2
    pad = np.zeros((C, H + 2 * r, W + 2 * r))
    pad[:, r:r + H, r:r + W] = a
    out = np.zeros((C, H, W))
    for di in range(w2.shape[0]):
        for dj in range(w2.shape[1]):
            out += w2[di, dj] * pad[:, di:di + H, dj:dj + W]
    return out


def ssim_stats(x: np.ndarray, y: np.ndarray) -> dict:
    """Window statistics and the SSIM map of x against y ([C][H][W])."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    w2 = window_2d()
    mx = _window_sum(x, w2)
    my = _window_sum(y, w2)
    exx = _window_sum(x * x, w2)
    eyy = _window_sum(y * y, w2)
    exy = _window_sum(x * y, w2)
    vx = exx - mx * mx
    vy = eyy - my * my
    cxy = exy - mx * my
    a1 = 2.0 * mx * my + C1
    a2 = 2.0 * cxy + C2
    b1 = mx * mx + my * my + C1
    b2 = vx + vy + C2
    s = (a1 * a2) / (b1 * b2)
    return dict(mx=mx, my=my, exx=exx, eyy=eyy, exy=exy, vx=vx, vy=vy, cxy=cxy,
                a1=a1, a2=a2, b1=b1, b2=b2, ssim=s)


def ssim_map(x, y) -> np.ndarray:
    return ssim_stats(x, y)["ssim"]


def loss(image, target, lam: float = LAMBDA, image_l1=None) -> dict:
    """Eq. 1 (image_l1 None) or Eq. 3 (L1 on image_l1 = I^a, D-SSIM on
    image = I^r).  Returns dict loss, l1, ssim (the means)."""
    x = np.asarray(image, np.float64)
    y = np.asarray(target, np.float64)
    xa = x if image_l1 is None else np.asarray(image_l1, np.float64)
    l1 = float(np.mean(np.abs(xa - y)))
    ssim = float(np.mean(ssim_map(x, y)))
    return dict(loss=(1.0 - lam) * l1 + lam * (1.0 - ssim), l1=l1, ssim=ssim)


def loss_grad(image, target, lam: float = LAMBDA, image_l1=None):
    """Gradient of `loss`.  Returns (d_image, d_image_l1): with image_l1
    None the second is None and d_image holds both terms."""
    x = np.asarray(image, np.float64)
    y = np.asarray(target, np.float64)
    n = x.size
    st = ssim_stats(x, y)
    # dLoss/dSSIM(p) for every pixel p of the map
    g = -lam / n
    mx, my, s = st["mx"], st["my"], st["ssim"]
    a1, a2, b1, b2 = st["a1"], st["a2"], st["b1"], st["b2"]
    # partials of SSIM(p) w.r.t. its window sums mu_x, E[x^2], E[xy]
    # (mu_y, E[y^2] belong to the target and carry no gradient)
    d_mx = g * (2.0 * my * (a2 - a1) / (b1 * b2) - 2.0 * mx * s * (1.0 / b1 - 1.0 / b2))
    d_exx = g * (-s / b2)
    d_exy = g * (2.0 * a1 / (b1 * b2))
    # adjoint of a zero-padded window sum with a symmetric window is the
    # same window sum of the adjoint field (zero outside the image)
    w2 = window_2d()
    dx = _window_sum(d_mx, w2) + 2.0 * x * _window_sum(d_exx, w2) + y * _window_sum(d_exy, w2)
    xa = x if image_l1 is None else np.asarray(image_l1, np.float64)
    dl1 = (1.0 - lam) / n * np.sign(xa - y)
    if image_l1 is None:
        return dx + dl1, None
    return dx, dl1
