"""Pins of the FP64 loss oracle (Eq. 1 and Eq. 3 of VastGaussian,
arXiv 2402.17427, sections 4.2 and 4.3: (1 - lambda) L1 + lambda D-SSIM).

Each test checks the oracle against something other than its own formulas:
properties that fix the Gaussian window, the closed form of SSIM for
constant images (border pixels included, where zero padding leaves part of
the window outside the image), the textbook weighted statistics of Wang et
al. evaluated by scalar loops at interior pixels, symmetry and the optimum,
central finite differences of the loss for the analytic gradient, and
planted mistakes that those pins must catch.
"""
import math

import numpy as np
import pytest

from gen import images
from oracle import loss as L


# ----------------------------------------------------------------- window --

def test_window_is_a_normalised_sampled_gaussian_of_sigma_1p5():
    g = L.window_1d()
    assert g.shape == (11,)
    assert abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g, g[::-1], rtol=0, atol=1e-18)
    # log-quadratic: g[k-1] g[k+1] / g[k]^2 = exp(-1 / sigma^2) for every k
    ratio = g[:-2] * g[2:] / g[1:-1] ** 2
    assert np.allclose(ratio, math.exp(-1.0 / 2.25), rtol=1e-13, atol=0)
    # second moment of the truncated sampled Gaussian: sigma^2 minus the
    # mass beyond +-5 (about 1e-3 of it)
    k = np.arange(11) - 5.0
    var = float((k * k * g).sum())
    assert 2.2 < var < 2.25


# ------------------------------------------------------- constant images --

def _partial_mass(n):
    """Window mass inside [0, n) for each position (1D, zero padding)."""
    g = L.window_1d()
    m = np.zeros(n)
    for i in range(n):
        for k in range(11):
            if 0 <= i + k - 5 < n:
                m[i] += g[k]
    return m


@pytest.mark.parametrize("a,b", [(0.7, 0.3), (0.2, 0.9), (0.5, 0.5), (0.0, 0.6)])
def test_constant_images_closed_form_including_borders(a, b):
    """x = a, y = b everywhere.  With w the window mass inside the image,
    mu_x = a w, E[x^2] = a^2 w, so sigma_x^2 = a^2 w (1 - w), sigma_xy =
    a b w (1 - w), and SSIM = (2ab w^2 + C1)(2ab w(1-w) + C2) /
    (((a^2 + b^2) w^2 + C1)((a^2 + b^2) w (1 - w) + C2)).  In the interior
    (w = 1) this is (2ab + C1) / (a^2 + b^2 + C1)."""
    H, W = 17, 23
    x = np.full((1, H, W), a)
    y = np.full((1, H, W), b)
    s = L.ssim_map(x, y)[0]
    w = np.outer(_partial_mass(H), _partial_mass(W))
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    want = ((2 * a * b * w * w + c1) * (2 * a * b * w * (1 - w) + c2)
            / (((a * a + b * b) * w * w + c1) * ((a * a + b * b) * w * (1 - w) + c2)))
    assert np.max(np.abs(s - want)) < 1e-12
    assert abs(s[8, 11] - (2 * a * b + c1) / (a * a + b * b + c1)) < 1e-12
    # the corner keeps (0.5 + g0 / 2)^2 of the window
    g0 = 1.0 / sum(math.exp(-k * k / 4.5) for k in range(-5, 6))
    assert abs(w[0, 0] - (0.5 + g0 / 2) ** 2) < 1e-15


# ---------------------------------------------- textbook statistics (Wang) --

def _ssim_textbook(x, y, i, j):
    """SSIM at one interior pixel from the weighted statistics of Wang et al.
    (2004): mu = sum w x, sigma^2 = sum w (x - mu)^2, sigma_xy = sum w (x -
    mu_x)(y - mu_y), scalar loops."""
    sig = 1.5
    w = [[math.exp(-((u - 5) ** 2 + (v - 5) ** 2) / (2 * sig * sig)) for v in range(11)] for u in range(11)]
    tot = sum(sum(r) for r in w)
    mx = my = 0.0
    for u in range(11):
        for v in range(11):
            mx += w[u][v] / tot * x[i + u - 5][j + v - 5]
            my += w[u][v] / tot * y[i + u - 5][j + v - 5]
    vx = vy = cxy = 0.0
    for u in range(11):
        for v in range(11):
            dx = x[i + u - 5][j + v - 5] - mx
            dy = y[i + u - 5][j + v - 5] - my
            vx += w[u][v] / tot * dx * dx
            vy += w[u][v] / tot * dy * dy
            cxy += w[u][v] / tot * dx * dy
    c1, c2 = 1e-4, 9e-4
    return (2 * mx * my + c1) * (2 * cxy + c2) / ((mx * mx + my * my + c1) * (vx + vy + c2))


def test_interior_pixels_match_the_textbook_weighted_statistics():
    r, t = images.image_pair(7, 31, 26, channels=2)
    s = L.ssim_map(r, t)
    for c in range(2):
        for (i, j) in [(5, 5), (12, 17), (20, 25), (9, 6), (13, 13)]:
            want = _ssim_textbook(r[c].astype(np.float64).tolist(), t[c].astype(np.float64).tolist(), i, j)
            assert abs(s[c, i, j] - want) < 1e-12


# ------------------------------------------------- symmetry and optimum --

def test_ssim_symmetry_and_optimum():
    r, t = images.image_pair(3, 20, 15)
    assert np.max(np.abs(L.ssim_map(r, t) - L.ssim_map(t, r))) < 1e-15
    assert np.max(np.abs(L.ssim_map(r, r) - 1.0)) < 1e-12
    out = L.loss(r, r)
    assert abs(out["loss"]) < 1e-12 and out["l1"] == 0.0
    d, _ = L.loss_grad(r, r)
    assert np.max(np.abs(d)) < 1e-14
    # structure differs: SSIM below 1 and the loss positive
    out = L.loss(r, t)
    assert out["ssim"] < 0.99 and out["loss"] > 0


def test_lambda_end_points():
    r, t = images.image_pair(4, 19, 14)
    r64, t64 = r.astype(np.float64), t.astype(np.float64)
    assert abs(L.loss(r, t, lam=0.0)["loss"] - np.abs(r64 - t64).mean()) < 1e-15
    assert abs(L.loss(r, t, lam=1.0)["loss"] - (1.0 - L.ssim_map(r, t).mean())) < 1e-15


# ------------------------------------------------------ gradient vs FD ----

def _fd_check(lam, eq3, seed, H=13, W=14, C=2):
    rng = np.random.default_rng(seed)
    r, t = images.image_pair(seed, W, H, channels=C)
    x = r.astype(np.float64)
    y = t.astype(np.float64)
    # keep |x - y| away from 0 so the L1 term is differentiable for the step
    x = np.where(np.abs(x - y) < 0.02, y + 0.05, x)
    xa = None
    if eq3:
        xa = y + rng.choice([-1.0, 1.0], y.shape) * rng.uniform(0.03, 0.2, y.shape)
    dx, dxa = L.loss_grad(x, y, lam=lam, image_l1=xa)
    h = 1e-6
    idx = [(0, 0, 0), (C - 1, H - 1, W - 1), (0, 6, 7), (C - 1, 0, W - 1), (0, H - 1, 3), (C - 1, 4, 0),
           (0, 2, 9)]
    scale = np.max(np.abs(dx))
    for (c, i, j) in idx:
        for which in ([0, 1] if eq3 else [0]):
            base = x if which == 0 else xa
            p = base.copy()
            m = base.copy()
            p[c, i, j] += h
            m[c, i, j] -= h
            if which == 0:
                fp = L.loss(p, y, lam, xa)["loss"]
                fm = L.loss(m, y, lam, xa)["loss"]
                an = dx[c, i, j]
            else:
                fp = L.loss(x, y, lam, p)["loss"]
                fm = L.loss(x, y, lam, m)["loss"]
                an = dxa[c, i, j]
            fd = (fp - fm) / (2 * h)
            assert abs(fd - an) < 1e-6 * scale + 1e-9 * abs(an), (lam, eq3, c, i, j, which, fd, an)


@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_gradient_matches_finite_differences_eq1(lam):
    _fd_check(lam, False, 21)


def test_gradient_matches_finite_differences_eq3():
    _fd_check(0.2, True, 22)


# ------------------------------------------------------- planted mistakes --

def test_pins_catch_planted_mistakes(monkeypatch):
    """A wrong constant and a dropped gradient factor must fail the pins
    above (the mistakes are planted in the oracle, on the CPU)."""
    x = np.full((1, 12, 12), 0.7)
    y = np.full((1, 12, 12), 0.3)
    good = L.ssim_map(x, y)[0, 0, 0]
    monkeypatch.setattr(L, "C2", 0.02 ** 2)
    assert abs(L.ssim_map(x, y)[0, 0, 0] - good) > 1e-4
    monkeypatch.setattr(L, "C2", 0.03 ** 2)
    real = L._window_sum

    def reflect_sum(a, w2):
        r = w2.shape[0] // 2
        pad = np.pad(a, ((0, 0), (r, r), (r, r)), mode="reflect")
        out = np.zeros(a.shape)
        for di in range(w2.shape[0]):
            for dj in range(w2.shape[1]):
                out += w2[di, dj] * pad[:, di:di + a.shape[1], dj:dj + a.shape[2]]
        return out

    monkeypatch.setattr(L, "_window_sum", reflect_sum)
    assert abs(L.ssim_map(x, y)[0, 0, 0] - good) > 1e-4
    monkeypatch.setattr(L, "_window_sum", real)
    # drop the 2 x factor of the E[x^2] term: the FD check must fail
    orig = L.loss_grad

    def bad_grad(image, target, lam=L.LAMBDA, image_l1=None):
        d, da = orig(image, target, lam, image_l1)
        st = L.ssim_stats(image, target)
        g = -lam / np.asarray(image).size
        dexx = L._window_sum(g * (-st["ssim"] / st["b2"]), L.window_2d())
        return d - np.asarray(image, np.float64) * dexx, da

    monkeypatch.setattr(L, "loss_grad", bad_grad)
    with pytest.raises(AssertionError):
        _fd_check(0.2, False, 21)
