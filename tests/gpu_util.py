"""Helpers for the GPU parity tests: unpacking the device projection record
and the gradient tolerance used across tests.

Tolerances (written out here once, used by every GPU test):
  image        |I_gpu - I_ref| <= 1e-4 at every pixel the oracle does not
               flag as ambiguous (a discontinuous decision within its
               window of the threshold); flagged pixels are counted, are at
               most 1e-3 of the pixels, and each is within 1/255 + 1e-4
               (one decision taken the other way changes the pixel by at
               most alpha T rgb with alpha at the 1/255 threshold).
  gradients    per parameter group, elementwise
               |g - g_ref| <= 1e-3 (|g_ref| + 1e-2 max|g_ref|_group)
               and ||g - g_ref|| / ||g_ref|| <= 1e-3, over the Gaussians that
               touch no flagged pixel.
  integers     keys, values, ranges, tile rectangles: bit-exact.
  optimiser    one step from the same FP32 state (adam_close): first moment
               within 6e-7 of the magnitudes of its two terms, second moment
               6e-7 relative, raw values 1.2e-7 relative plus the update's
               error, activated scale and opacity through exp and sigmoid.
"""
from __future__ import annotations

import numpy as np

IMAGE_ATOL = 1e-4
GRAD_RTOL = 1e-3
GRAD_FLOOR = 1e-2


def unpack_rec(rec_f32: np.ndarray, n: int) -> dict:
    """Split the 48-byte device records (as a float32 array) into fields."""
    raw = np.ascontiguousarray(rec_f32[: n * 12]).view(np.uint8).reshape(n, 48)
    uv = raw[:, 0:16].copy().view(np.float64).reshape(n, 2)
    f = raw[:, 16:48].copy().view(np.float32).reshape(n, 8)
    return dict(uv=uv, conic=f[:, 0:3].astype(np.float64), opacity=f[:, 3].astype(np.float64),
                rgb=f[:, 4:7].astype(np.float64), thr=f[:, 7].astype(np.float64))


def grad_close(name, g, ref, rtol=GRAD_RTOL, floor=GRAD_FLOOR):
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    assert g.shape == ref.shape, (name, g.shape, ref.shape)
    if ref.size == 0:
        return 0.0
    scale = np.abs(ref).max()
    err = np.abs(g - ref)
    lim = rtol * (np.abs(ref) + floor * scale)
    bad = err > lim
    nrm = np.linalg.norm(ref)
    rel = np.linalg.norm(g - ref) / nrm if nrm > 0 else np.linalg.norm(g)
    if bad.any() or rel > rtol:
        i = np.unravel_index(np.argmax(err - lim), err.shape)
        raise AssertionError(f"{name}: {bad.sum()} of {bad.size} elements outside tolerance, norm rel {rel:.3e}; "
                             f"worst at {i}: got {g[i]:.6e} want {ref[i]:.6e} (scale {scale:.3e})")
    return rel


FLAGGED_ATOL = 1.0 / 255.0 + 1e-4
MAX_FLAGGED_FRAC = 1e-3


def image_close(name, img, ref, flags, atol=IMAGE_ATOL, max_flagged_frac=MAX_FLAGGED_FRAC):
    """Image parity: `img` and `ref` are [3][...] (or [...] for a plane),
    `flags` the oracle's per-pixel flags; bit 0 marks an image decision near
    its threshold (bit 1, an alpha near the 0.99 cap, changes only the
    gradient).  Returns (worst error at unflagged pixels, number of flagged
    pixels, worst error at flagged pixels)."""
    img = np.asarray(img, np.float64)
    ok = (np.asarray(flags) & 1) == 0
    diff = np.abs(img - ref)
    chan = diff.ndim == ok.ndim + 1          # leading channel axis
    err = diff[:, ok] if chan else diff[ok]
    worst = float(err.max()) if err.size else 0.0
    assert worst <= atol, f"{name}: max error {worst:.3e} at unflagged pixels (atol {atol})"
    ferr = diff[:, ~ok] if chan else diff[~ok]
    fworst = float(ferr.max()) if ferr.size else 0.0
    nflag = int((~ok).sum())
    print(f"[image] {name}: max err {worst:.2e} unflagged, {nflag} flagged pixels (max err {fworst:.2e})",
          flush=True)
    assert fworst <= FLAGGED_ATOL, f"{name}: a flagged pixel is off by {fworst:.3e} (bound {FLAGGED_ATOL:.3e})"
    frac = float((~ok).mean())
    assert frac <= max_flagged_frac, f"{name}: {frac:.4f} of pixels flagged"
    return worst, nflag, fworst


def adam_close(pre_raw, pre_m, pre_v, grad_act, got, hyper, deg, step):
    """One Adam step of the FP64 oracle from the FP32 state (planes
    [11 + 3K][n]) against the kernel's result `got` (dict raw, m, v, scale,
    opacity; same planes, scale [3][n], opacity [n])."""
    from oracle import adam as A
    raw, g, m0, v0 = (np.asarray(a, np.float64) for a in (pre_raw, grad_act, pre_m, pre_v))
    cfg = {k: float(np.float32(v)) for k, v in hyper.items()}
    r1, m1, v1 = A.adam_step(raw, m0, v0, g, cfg, deg, step)
    graw = A.raw_gradient(raw, g)
    b1 = cfg["beta1"]
    tol_m = 6e-7 * (b1 * np.abs(m0) + (1 - b1) * np.abs(graw)) + 1e-37
    err = np.abs(got["m"] - m1)
    assert np.all(err <= tol_m), ("m", np.max(err / tol_m))
    assert np.all(np.abs(got["v"] - v1) <= 6e-7 * v1 + 1e-37), "v"
    lr = A.lr_of_planes(cfg, deg)[:, None]
    ss = lr / (1 - cfg["beta1"] ** step)
    den = np.sqrt(v1 / (1 - cfg["beta2"] ** step)) + cfg["eps"]
    tol_r = 1.2e-7 * np.abs(r1) + ss * (tol_m + 1e-6 * np.abs(m1)) / den + 1e-30
    err = np.abs(got["raw"] - r1)
    assert np.all(err <= tol_r), ("raw", np.unravel_index(np.argmax(err / tol_r), err.shape), np.max(err / tol_r))
    act = A.activated(r1)
    assert np.all(np.abs(got["scale"] - act["scale"]) <= act["scale"] * (3e-7 + 1.0001 * tol_r[3:6]) + 1e-38), "scale"
    o = act["opacity"]
    assert np.all(np.abs(got["opacity"] - o) <= 3e-7 * o + o * (1 - o) * tol_r[10] + 1e-38), "opacity"
