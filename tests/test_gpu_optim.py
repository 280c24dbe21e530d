"""GPU parity of the optimiser step (gs_adam_step: Adam over the raw
Gaussian properties with the 3DGS activations, and the densification
statistics) against the FP64 oracle.

Every test calls the HIP kernel through the C ABI on seeded FP32 state and
gives the oracle the same FP32 values.  Tolerances, for one step from the
same inputs (FP32 arithmetic, a few roundings per element):
  m        |dm| <= 6e-7 (beta1 |m0| + (1 - beta1) |g|)   (terms may cancel)
  v        relative 6e-7
  raw      1.2e-7 |raw| (its own rounding) plus the update's error: step
           size times (the m bound + 1e-6 |m|) / denominator
  scale    relative 3e-7 plus scale times the raw bound (exp)
  opacity  3e-7 opacity plus o (1 - o) times the raw bound (sigmoid)
  accum    relative 3e-7; visible_count exact.
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adam as A
from paper_2402_17427_amd import _native as N
from paper_2402_17427_amd import optim
from paper_2402_17427_amd.raster import _ptr

from gpu_util import adam_close

pytestmark = pytest.mark.gpu

HYPER = dict(optim.DEFAULTS, lr_mean=3e-4)


def _case(name):
    print(f"\n[case] {name}", flush=True)


def _f32(a):
    return np.ascontiguousarray(a, np.float32)


def _dev(a):
    return torch.as_tensor(_f32(a)).cuda()


def _state(seed, n, deg, ld=None, fresh=False):
    K = (deg + 1) ** 2
    P = 11 + 3 * K
    ld = n if ld is None else ld
    rng = np.random.default_rng(seed)
    raw = rng.normal(0, 1, (P, ld)).astype(np.float32)
    raw[3:6] = rng.normal(-3, 1, (3, ld))           # log-scales
    raw[10] = rng.normal(0, 2, ld)                   # logits
    g = (rng.normal(0, 1e-4, (P, ld)) * (rng.uniform(size=(P, ld)) > 0.25)).astype(np.float32)
    if fresh:
        m = np.zeros((P, ld), np.float32)
        v = np.zeros((P, ld), np.float32)
    else:
        m = rng.normal(0, 1e-5, (P, ld)).astype(np.float32)
        v = (rng.normal(0, 1e-4, (P, ld)) ** 2).astype(np.float32)
    g2d = rng.normal(0, 1e-6, (9, max(n, 1))).astype(np.float32)
    tiles = (rng.integers(0, 5, max(n, 1)) * (rng.uniform(size=max(n, 1)) > 0.3)).astype(np.int32)
    acc = rng.uniform(0, 1e-4, ld).astype(np.float32)
    cnt = rng.integers(0, 50, ld).astype(np.float32)
    return dict(raw=raw, g=g, m=m, v=v, g2d=g2d, tiles=tiles, acc=acc, cnt=cnt, K=K, P=P, ld=ld)


def _run(s, n, deg, step, status=0, stats=True):
    """Upload the state, run one gs_adam_step, return the device results."""
    K, ld = s["K"], s["ld"]
    raw = s["raw"]
    d = {k: _dev(raw[a:b]) for k, (a, b) in dict(mean=(0, 3), ls=(3, 6), quat=(6, 10), lo=(10, 11),
                                                    sh=(11, 11 + 3 * K)).items()}
    scale_out = _dev(np.exp(raw[3:6].astype(np.float64)))
    op_out = _dev(1 / (1 + np.exp(-raw[10].astype(np.float64))))
    gd = _dev(s["g"])
    m, v = _dev(s["m"]), _dev(s["v"])
    acc, cnt = _dev(s["acc"]), _dev(s["cnt"])
    g2d = _dev(s["g2d"])
    tiles = torch.as_tensor(s["tiles"]).cuda()
    st = torch.tensor([status], dtype=torch.int32).cuda()
    p = N.gs_params()
    p.n, p.ld, p.sh_degree = n, ld, deg
    p.mean, p.log_scale, p.quat, p.logit_opacity, p.sh = (_ptr(d["mean"]), _ptr(d["ls"]), _ptr(d["quat"]),
                                                          _ptr(d["lo"]), _ptr(d["sh"]))
    gr = N.gs_grads()
    gr.ld = ld
    gr.mean, gr.scale, gr.quat = _ptr(gd[0:3]), C.c_void_p(gd.data_ptr() + 3 * ld * 4), \
        C.c_void_p(gd.data_ptr() + 6 * ld * 4)
    gr.opacity, gr.sh = C.c_void_p(gd.data_ptr() + 10 * ld * 4), C.c_void_p(gd.data_ptr() + 11 * ld * 4)
    gr.grad2d = _ptr(g2d)
    stt = N.gs_adam_state()
    stt.m, stt.v, stt.grad_accum, stt.visible_count = _ptr(m), _ptr(v), _ptr(acc), _ptr(cnt)
    cfg = optim.config(step, **HYPER)
    N.call("gs_adam_step", C.byref(p), _ptr(scale_out), _ptr(op_out), C.byref(stt), C.byref(gr),
           _ptr(tiles) if stats else None, _ptr(st), C.byref(cfg), None)
    torch.cuda.synchronize()
    out_raw = np.concatenate([d["mean"].cpu().numpy(), d["ls"].cpu().numpy(), d["quat"].cpu().numpy(),
                              d["lo"].cpu().numpy(), d["sh"].cpu().numpy()], axis=0)
    return dict(raw=out_raw, m=m.cpu().numpy(), v=v.cpu().numpy(), scale=scale_out.cpu().numpy(),
                opacity=op_out.cpu().numpy(), acc=acc.cpu().numpy(), cnt=cnt.cpu().numpy())


def _check(s, got, n, deg, step):
    g = {k: (v[..., :n]) for k, v in got.items() if k in ("raw", "m", "v", "scale", "opacity")}
    adam_close(s["raw"][:, :n], s["m"][:, :n], s["v"][:, :n], s["g"][:, :n], g, HYPER, deg, step)


@pytest.mark.parametrize("n,deg,step,fresh", [(1000, 3, 1, True), (4099, 3, 7, False), (1, 0, 2, False),
                                               (1500, 1, 30, False), (1025, 2, 3, False)])
def test_adam_step_matches_the_oracle(n, deg, step, fresh):
    _case(f"adam n={n} deg={deg} step={step}")
    s = _state(n + deg, n, deg, fresh=fresh)
    got = _run(s, n, deg, step)
    _check(s, got, n, deg, step)
    acc, cnt = A.densify_stats(s["acc"][:n], s["cnt"][:n], (s["g2d"][0, :n], s["g2d"][1, :n]),
                               s["tiles"][:n] > 0)
    np.testing.assert_allclose(got["acc"][:n], acc, rtol=3e-7, atol=1e-38)
    np.testing.assert_array_equal(got["cnt"][:n], cnt)


def test_stride_padding_is_left_alone_and_no_stats_without_visibility():
    _case("adam ld > n, no statistics")
    n, ld, deg = 777, 1024, 3
    s = _state(5, n, deg, ld=ld)
    got = _run(s, n, deg, 4, stats=False)
    _check(s, got, n, deg, 4)
    for k in ("raw", "m", "v"):
        np.testing.assert_array_equal(got[k][:, n:], s[k][:, n:])
    np.testing.assert_array_equal(got["acc"], s["acc"])
    np.testing.assert_array_equal(got["cnt"], s["cnt"])


def test_status_flag_skips_the_step():
    """A step whose bins overflowed has no valid gradient: nothing moves."""
    _case("adam status set")
    n, deg = 2000, 3
    s = _state(6, n, deg)
    got = _run(s, n, deg, 3, status=N.GS_ERR_CAPACITY)
    for k in ("raw", "m", "v"):
        np.testing.assert_array_equal(got[k], s[k])
    np.testing.assert_array_equal(got["acc"], s["acc"])


def test_full_size_cell_one_million_gaussians():
    """The bench's cell size (1M Gaussians, SH degree 3), every element."""
    _case("adam 1M SH3")
    n, deg = 1_000_000, 3
    s = _state(7, n, deg)
    got = _run(s, n, deg, 11)
    _check(s, got, n, deg, 11)
    acc, cnt = A.densify_stats(s["acc"], s["cnt"], (s["g2d"][0], s["g2d"][1]), s["tiles"] > 0)
    np.testing.assert_allclose(got["acc"], acc, rtol=3e-7, atol=1e-38)
    np.testing.assert_array_equal(got["cnt"], cnt)
