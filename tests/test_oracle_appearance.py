"""Pins of the FP64 appearance-model oracle (VastGaussian, arXiv 2402.17427,
section 4.2 and supplement S1.1): every layer against PyTorch's CPU
implementation of the same operation (convolution, pixel shuffle, bilinear
interpolation with half-pixel centres), the block downsampling against
scalar loops, the whole forward and backward against PyTorch autograd in
float64, and a planted layer mistake that the comparison catches.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
F = torch.nn.functional

from oracle import appearance as A


def _params(seed, embed=A.EMBED, scale=0.05):
    rng = np.random.default_rng(seed)
    return [(rng.normal(0, scale, (co, ci, 3, 3)), rng.normal(0, 0.02, co)) for co, ci in A.layer_shapes(embed)]


def test_downsample_by_loops():
    rng = np.random.default_rng(1)
    img = rng.uniform(0, 1, (3, 70, 45))
    d = A.downsample(img)
    assert d.shape == (3, 3, 2)
    for c in range(3):
        for y in range(3):
            for x in range(2):
                s, n = 0.0, 0
                for yy in range(y * 32, min(y * 32 + 32, 70)):
                    for xx in range(x * 32, min(x * 32 + 32, 45)):
                        s += img[c, yy, xx]
                        n += 1
                assert abs(d[c, y, x] - s / n) < 1e-14
    # adjoint: <A x, g> = <x, A^T g>
    g = rng.normal(size=d.shape)
    assert abs((d * g).sum() - (img * A.downsample_adjoint(g, 70, 45)).sum()) < 1e-12


def test_layers_match_pytorch():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(8, 9, 11))
    w = rng.normal(size=(5, 8, 3, 3))
    b = rng.normal(size=5)
    ref = F.conv2d(torch.tensor(x)[None], torch.tensor(w), torch.tensor(b), padding=1)[0].numpy()
    np.testing.assert_allclose(A.conv3x3(x, w, b), ref, rtol=1e-12, atol=1e-12)
    ref = F.pixel_shuffle(torch.tensor(x)[None], 2)[0].numpy()
    np.testing.assert_array_equal(A.pixel_shuffle(x), ref)
    for (H, W) in [(18, 22), (31, 17), (40, 70)]:
        ref = F.interpolate(torch.tensor(x)[None], size=(H, W), mode="bilinear", align_corners=False)[0].numpy()
        np.testing.assert_allclose(A.bilinear(x, H, W), ref, rtol=1e-12, atol=1e-12)


def _torch_model(img, embed, params):
    """The same network with PyTorch CPU operations (float64, autograd)."""
    t = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)
    ti, te = t(img), t(embed)
    tp = [(t(w), t(b)) for w, b in params]
    C, H, W = img.shape
    h, w = -(-H // 32), -(-W // 32)
    # block means with partial border blocks, as explicit sums
    rows = []
    for y in range(h):
        cols = []
        for x in range(w):
            cols.append(ti[:, y * 32:(y + 1) * 32, x * 32:(x + 1) * 32].mean(dim=(1, 2)))
        rows.append(torch.stack(cols, dim=1))
    d = torch.stack(rows, dim=1)
    D = torch.cat([d, te[:, None, None].expand(len(embed), h, w)], dim=0)[None]
    x = F.conv2d(D, tp[0][0], tp[0][1], padding=1)
    for k in range(1, 5):
        x = F.relu(F.conv2d(F.pixel_shuffle(x, 2), tp[k][0], tp[k][1], padding=1))
    u = F.interpolate(x, size=(H, W), mode="bilinear", align_corners=False)
    f1 = F.relu(F.conv2d(u, tp[5][0], tp[5][1], padding=1))
    M = F.conv2d(f1, tp[6][0], tp[6][1], padding=1)[0]
    return ti, te, tp, M, ti * M


def _compare(seed, H, W, embed_len=A.EMBED):
    rng = np.random.default_rng(seed)
    img = rng.uniform(0, 1, (3, H, W))
    emb = rng.normal(0, 1, embed_len)
    params = _params(seed + 1, embed_len)
    M, Ia, cache = A.forward(img, emb, params)
    ti, te, tp, tM, tIa = _torch_model(img, emb, params)
    np.testing.assert_allclose(M, tM.detach().numpy(), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(Ia, tIa.detach().numpy(), rtol=1e-10, atol=1e-12)
    g = rng.normal(0, 1, (3, H, W))
    (tIa * torch.tensor(g)).sum().backward()
    d_img, d_emb, grads = A.backward(img, emb, params, cache, M, g)
    np.testing.assert_allclose(d_img, ti.grad.numpy(), rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(d_emb, te.grad.numpy(), rtol=1e-9, atol=1e-11)
    for k in range(7):
        np.testing.assert_allclose(grads[k][0], tp[k][0].grad.numpy(), rtol=1e-9, atol=1e-11)
        np.testing.assert_allclose(grads[k][1], tp[k][1].grad.numpy(), rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("seed,H,W", [(3, 70, 100), (4, 64, 64), (5, 33, 95)])
def test_forward_and_backward_match_pytorch_autograd(seed, H, W):
    _compare(seed, H, W)


def test_planted_pixel_shuffle_order_is_caught(monkeypatch):
    """Channel order c + C (2i + j) instead of 4c + 2i + j (a plausible
    slip) must fail the comparison (planted in the oracle, on the CPU)."""
    def wrong(x):
        C4, h, w = x.shape
        C = C4 // 4
        out = np.zeros((C, 2 * h, 2 * w))
        for i in range(2):
            for j in range(2):
                out[:, i::2, j::2] = x[[c + C * (2 * i + j) for c in range(C)]]
        return out

    monkeypatch.setattr(A, "pixel_shuffle", wrong)
    with pytest.raises(AssertionError):
        _compare(3, 70, 100)
