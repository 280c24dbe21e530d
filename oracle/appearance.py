"""FP64 CPU oracle for the decoupled appearance model -- TEST INFRASTRUCTURE.

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's `cpu_baseline`
leg may import this module; the GPU kernels share nothing with it.

What it computes (VastGaussian, arXiv 2402.17427, section 4.2 and
supplement S1.1): the rendered image I^r ([3][H][W]) is downsampled 32
times, an appearance embedding of length m (64) is concatenated to every
pixel of it, and a CNN turns the (3 + m)-channel map into a transformation
map M of the image's size; the appearance-adjusted image is the pixel-wise
product I^a = I^r * M.  The CNN: a 3x3 convolution to 256 channels, four
upsampling blocks (pixel shuffle by 2, 3x3 convolution that halves the
channels of the block input, ReLU), bilinear interpolation to H x W, a 3x3
convolution, ReLU, and a 3x3 convolution to 3 channels.
Readings where the paper is silent:
  * the downsampled map has ceil(H/32) x ceil(W/32) pixels, each the mean of
    the image pixels of its 32 x 32 block (border blocks over the pixels
    they hold); the gradient flows through it into I^r;
  * every convolution has a bias, zero padding 1 and stride 1; the first
    convolution has no activation, the last none either (M is used as is);
    the convolution after the interpolation keeps 16 channels;
  * pixel shuffle: out[c][2y + i][2x + j] = in[4c + 2i + j][y][x];
  * bilinear interpolation with half-pixel centres (source coordinate
    (d + 0.5) * in / out - 0.5, clamped below at 0, the upper neighbour
    clamped at the last pixel).
Layer parameters are given as a list of (weight [Cout][Cin][3][3], bias
[Cout]) in the order conv0, the four block convolutions, the two final
convolutions.  Everything is float64.
"""
from __future__ import annotations

import numpy as np

EMBED = 64
DOWN = 32


def layer_shapes(embed=EMBED):
    """(Cout, Cin) of the seven convolutions."""
    return [(256, 3 + embed), (128, 64), (64, 32), (32, 16), (16, 8), (16, 16), (3, 16)]


def downsample(img):
    C, H, W = img.shape
    h, w = -(-H // DOWN), -(-W // DOWN)
    out = np.zeros((C, h, w))
    for y in range(h):
        for x in range(w):
            blk = img[:, y * DOWN:(y + 1) * DOWN, x * DOWN:(x + 1) * DOWN]
            out[:, y, x] = blk.reshape(C, -1).mean(axis=1)
    return out


def downsample_adjoint(g, H, W):
    C, h, w = g.shape
    out = np.zeros((C, H, W))
    for y in range(h):
        for x in range(w):
            ys, xs = slice(y * DOWN, min((y + 1) * DOWN, H)), slice(x * DOWN, min((x + 1) * DOWN, W))
            cnt = (ys.stop - ys.start) * (xs.stop - xs.start)
            out[:, ys, xs] += g[:, y, x][:, None, None] / cnt
    return out


def conv3x3(x, wgt, b):
    """out[o][y][x] = b[o] + sum_{i, dy, dx} w[o][i][dy][dx] x[i][y+dy-1][x+dx-1]."""
    C, H, W = x.shape
    pad = np.zeros((C, H + 2, W + 2))
    pad[:, 1:-1, 1:-1] = x
    out = np.zeros((wgt.shape[0], H, W)) + b[:, None, None]
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("oi,ihw->ohw", wgt[:, :, dy, dx], pad[:, dy:dy + H, dx:dx + W])
    return out


def conv3x3_backward(x, wgt, gout):
    """(dx, dw, db) of conv3x3 for the output gradient gout."""
    C, H, W = x.shape
    pad = np.zeros((C, H + 2, W + 2))
    pad[:, 1:-1, 1:-1] = x
    dw = np.zeros_like(wgt)
    dpad = np.zeros_like(pad)
    for dy in range(3):
        for dx in range(3):
            dw[:, :, dy, dx] = np.einsum("ohw,ihw->oi", gout, pad[:, dy:dy + H, dx:dx + W])
            dpad[:, dy:dy + H, dx:dx + W] += np.einsum("oi,ohw->ihw", wgt[:, :, dy, dx], gout)
    return dpad[:, 1:-1, 1:-1], dw, gout.sum(axis=(1, 2))


def pixel_shuffle(x):
    C4, h, w = x.shape
    C = C4 // 4
    out = np.zeros((C, 2 * h, 2 * w))
    for i in range(2):
        for j in range(2):
            out[:, i::2, j::2] = x[[4 * c + 2 * i + j for c in range(C)]]
    return out


def pixel_shuffle_adjoint(g):
    C, H2, W2 = g.shape
    out = np.zeros((4 * C, H2 // 2, W2 // 2))
    for i in range(2):
        for j in range(2):
            out[[4 * c + 2 * i + j for c in range(C)]] = g[:, i::2, j::2]
    return out


def _bilinear_weights(n_in, n_out):
    """[n_out][n_in] interpolation matrix with half-pixel centres."""
    A = np.zeros((n_out, n_in))
    for d in range(n_out):
        s = max((d + 0.5) * n_in / n_out - 0.5, 0.0)
        i0 = min(int(np.floor(s)), n_in - 1)
        i1 = min(i0 + 1, n_in - 1)
        f = s - i0
        A[d, i0] += 1.0 - f
        A[d, i1] += f
    return A


def bilinear(x, H, W):
    """Ay x Ax^T per channel (rows, then columns)."""
    Ay = _bilinear_weights(x.shape[1], H)
    Ax = _bilinear_weights(x.shape[2], W)
    return np.stack([Ay @ x[c] @ Ax.T for c in range(x.shape[0])])


def bilinear_adjoint(g, h, w):
    """Ay^T g Ax per channel."""
    Ay = _bilinear_weights(h, g.shape[1])
    Ax = _bilinear_weights(w, g.shape[2])
    return np.stack([Ay.T @ g[c] @ Ax for c in range(g.shape[0])])


def forward(img, embed, params):
    """Returns (M, I^a, cache)."""
    img = np.asarray(img, np.float64)
    C, H, W = img.shape
    d = downsample(img)
    D = np.concatenate([d, np.broadcast_to(np.asarray(embed, np.float64)[:, None, None],
                                           (len(embed),) + d.shape[1:])], axis=0)
    cache = dict(D=D, H=H, W=W)
    x = conv3x3(D, *params[0])
    cache["x0"] = x
    for k in range(1, 5):
        s = pixel_shuffle(x)
        cache[f"s{k}"] = s
        x = np.maximum(conv3x3(s, *params[k]), 0.0)
        cache[f"x{k}"] = x
    u = bilinear(x, H, W)
    cache["u"] = u
    f1 = np.maximum(conv3x3(u, *params[5]), 0.0)
    cache["f1"] = f1
    M = conv3x3(f1, *params[6])
    return M, img * M, cache


def backward(img, embed, params, cache, M, d_adj):
    """Gradients of a loss whose gradient w.r.t. I^a is d_adj: returns
    (d_img, d_embed, [(dw, db)] per layer).  d_img includes both the
    multiplication and the path through the downsampling."""
    img = np.asarray(img, np.float64)
    d_adj = np.asarray(d_adj, np.float64)
    H, W = cache["H"], cache["W"]
    d_img = d_adj * M
    g = d_adj * img                      # dL/dM
    grads = [None] * 7
    g, dw, db = conv3x3_backward(cache["f1"], params[6][0], g)
    grads[6] = (dw, db)
    g = g * (cache["f1"] > 0)
    g, dw, db = conv3x3_backward(cache["u"], params[5][0], g)
    grads[5] = (dw, db)
    g = bilinear_adjoint(g, cache["x4"].shape[1], cache["x4"].shape[2])
    for k in range(4, 0, -1):
        g = g * (cache[f"x{k}"] > 0)
        g, dw, db = conv3x3_backward(cache[f"s{k}"], params[k][0], g)
        grads[k] = (dw, db)
        g = pixel_shuffle_adjoint(g)
    g, dw, db = conv3x3_backward(cache["D"], params[0][0], g)
    grads[0] = (dw, db)
    d_embed = g[3:].sum(axis=(1, 2))
    d_img = d_img + downsample_adjoint(g[:3], H, W)
    return d_img, d_embed, grads
