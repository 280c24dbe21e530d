"""Pins of the FP64 optimiser oracle (Adam over the raw Gaussian properties
with the 3DGS activations, and the densification statistics; VastGaussian,
arXiv 2402.17427, section 3 and section 5.1).

The oracle is checked against an independent implementation (PyTorch's
Adam, with the chain rule through exp and sigmoid taken by autograd), the
closed form of the first Adam step, hand-computed statistics, and planted
mistakes that the comparison must catch.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adam as A

CFG = dict(A.DEFAULTS, lr_mean=1e-3)


def _groups_torch(raw, K):
    """Raw planes -> named leaf tensors (SH DC and rest split)."""
    t = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)
    sh = raw[11:].reshape(3, K, -1)
    return dict(mean=t(raw[0:3]), scale=t(raw[3:6]), quat=t(raw[6:10]), opacity=t(raw[10:11]),
                sh_dc=t(sh[:, 0]), sh_rest=t(sh[:, 1:]))


def _planes_from(d, K):
    sh = np.concatenate([d["sh_dc"][:, None], d["sh_rest"]], axis=1).reshape(3 * K, -1)
    return np.concatenate([d["mean"], d["scale"], d["quat"], d["opacity"], sh], axis=0)


@pytest.mark.parametrize("deg", [0, 1, 3])
def test_adam_matches_torch_adam_with_autograd_chain_rule(deg):
    K = (deg + 1) ** 2
    P = 11 + 3 * K
    n = 37
    rng = np.random.default_rng(10 + deg)
    raw = rng.normal(0, 1, (P, n))
    leaves = _groups_torch(raw, K)
    groups = [dict(params=[leaves[k]], lr=CFG["lr_" + k]) for k in ("mean", "scale", "quat", "opacity", "sh_dc",
                                                                     "sh_rest") if leaves[k].numel() > 0]
    opt = torch.optim.Adam(groups, betas=(CFG["beta1"], CFG["beta2"]), eps=CFG["eps"])
    m = np.zeros((P, n))
    v = np.zeros((P, n))
    r = raw.copy()
    for step in range(1, 5):
        ga = rng.normal(0, 1e-3, (P, n)) * (rng.uniform(size=(P, n)) > 0.2)
        # autograd: L = sum(ga * activated(raw))
        opt.zero_grad()
        gsh = ga[11:].reshape(3, K, n)
        L = ((torch.tensor(ga[0:3]) * leaves["mean"]).sum()
             + (torch.tensor(ga[3:6]) * torch.exp(leaves["scale"])).sum()
             + (torch.tensor(ga[6:10]) * leaves["quat"]).sum()
             + (torch.tensor(ga[10:11]) * torch.sigmoid(leaves["opacity"])).sum()
             + (torch.tensor(gsh[:, 0]) * leaves["sh_dc"]).sum())
        if K > 1:
            L = L + (torch.tensor(gsh[:, 1:]) * leaves["sh_rest"]).sum()
        L.backward()
        opt.step()
        r, m, v = A.adam_step(r, m, v, ga, CFG, deg, step)
        got = _planes_from({k: t.detach().numpy() for k, t in leaves.items()}, K)
        np.testing.assert_allclose(r, got, rtol=1e-12, atol=1e-15)
        st = {k: opt.state[leaves[k]] for k in leaves if leaves[k].numel() > 0}
        if K == 1:
            st["sh_rest"] = dict(exp_avg=torch.zeros(3, 0, n), exp_avg_sq=torch.zeros(3, 0, n))
        gm = _planes_from({k: st[k]["exp_avg"].numpy() for k in leaves}, K)
        gv = _planes_from({k: st[k]["exp_avg_sq"].numpy() for k in leaves}, K)
        np.testing.assert_allclose(m, gm, rtol=1e-12, atol=1e-20)
        np.testing.assert_allclose(v, gv, rtol=1e-12, atol=1e-30)


def test_first_step_closed_form():
    """t = 1: m_hat = g, v_hat = g^2, so p1 = p0 - lr g / (|g| + eps)."""
    deg = 0
    P = 14
    rng = np.random.default_rng(3)
    raw = rng.normal(0, 1, (P, 9))
    ga = rng.normal(0, 1e-2, (P, 9))
    g = ga.copy()
    g[3:6] *= np.exp(raw[3:6])
    o = 1 / (1 + np.exp(-raw[10]))
    g[10] *= o * (1 - o)
    lr = np.array([CFG["lr_mean"]] * 3 + [CFG["lr_scale"]] * 3 + [CFG["lr_quat"]] * 4 + [CFG["lr_opacity"]]
                  + [CFG["lr_sh_dc"]] * 3)[:, None]
    want = raw - lr * g / (np.abs(g) + CFG["eps"])
    r, m, v = A.adam_step(raw, np.zeros_like(raw), np.zeros_like(raw), ga, CFG, deg, 1)
    np.testing.assert_allclose(r, want, rtol=1e-14, atol=1e-16)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_zero_gradient_still_moves_through_the_first_moment():
    P = 14
    raw = np.zeros((P, 2))
    ga = np.zeros((P, 2))
    ga[0] = [1e-3, -2e-3]
    r1, m1, v1 = A.adam_step(raw, np.zeros_like(raw), np.zeros_like(raw), ga, CFG, 0, 1)
    r2, m2, v2 = A.adam_step(r1, m1, v1, np.zeros_like(raw), CFG, 0, 2)
    # second step: m = 0.9 m1, v = 0.999 v1; moves by lr m_hat / sqrt(v_hat)
    m_hat = 0.9 * m1[0] / (1 - 0.9 ** 2)
    v_hat = 0.999 * v1[0] / (1 - 0.999 ** 2)
    np.testing.assert_allclose(r2[0] - r1[0], -CFG["lr_mean"] * m_hat / (np.sqrt(v_hat) + CFG["eps"]), rtol=1e-12)
    assert np.all(r2[1:] == 0.0)


def test_densify_stats_by_hand():
    acc = np.array([0.0, 1.0, 2.0, 0.5])
    cnt = np.array([0.0, 3.0, 1.0, 7.0])
    gu = np.array([3.0, -6.0, 1.0, 9.0])
    gv = np.array([4.0, 8.0, 0.0, 9.0])
    vis = np.array([True, True, False, True])
    a, c = A.densify_stats(acc, cnt, (gu, gv), vis)
    np.testing.assert_allclose(a, [5.0, 11.0, 2.0, 0.5 + 9.0 * math.sqrt(2.0)], rtol=1e-15)
    np.testing.assert_array_equal(c, [1.0, 4.0, 1.0, 8.0])


def test_planted_missing_bias_correction_is_caught(monkeypatch):
    """Dropping the bias correction (a plausible slip) must fail the
    comparison with PyTorch's Adam (planted in the oracle, on the CPU)."""
    real = A.adam_step

    def no_bias(raw, m, v, grad_act, cfg, sh_degree, step):
        g = A.raw_gradient(raw, grad_act)
        m = cfg["beta1"] * m + (1 - cfg["beta1"]) * g
        v = cfg["beta2"] * v + (1 - cfg["beta2"]) * g * g
        lr = A.lr_of_planes(cfg, sh_degree)[:, None]
        return raw - lr * m / (np.sqrt(v) + cfg["eps"]), m, v

    monkeypatch.setattr(A, "adam_step", no_bias)
    with pytest.raises(AssertionError):
        test_adam_matches_torch_adam_with_autograd_chain_rule(1)
    monkeypatch.setattr(A, "adam_step", real)
