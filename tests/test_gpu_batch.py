"""Batched cells (one persistent, graph-captured training step over several
cells of uneven sizes) against the plain single-view path and the oracle.
Each cell's image must be bit-identical to the plain path's, its L1 loss
equal to mean |I - I*|, and its gradients within tolerance of the plain
path's; graph replays must repeat the eager result."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from gen import scenes
from paper_2402_17427_amd import raster
from paper_2402_17427_amd.batch import BatchStep

from gpu_util import grad_close, image_close

pytestmark = pytest.mark.gpu

PARAMS = ("mean", "scale", "quat", "opacity", "sh")


def _case(name):
    print(f"\n[case] {name}", flush=True)


def _cells():
    specs = [(6_000, 21, 97, 61), (20_000, 22, 200, 150), (12_000, 23, 160, 96)]
    out = []
    for n, seed, w, h in specs:
        g, cam = scenes.small_city(n=n, seed=seed, width=w, height=h)
        tgt = np.random.default_rng(seed + 100).uniform(0, 1, (3, h, w)).astype(np.float32)
        out.append((g, cam, tgt))
    return out


def _plain(g, cam, tgt, tile):
    dg = raster.DeviceGaussians.from_host(g)
    f = raster.render(dg, cam, tile=tile)
    img = f.image.clone()
    t = torch.as_tensor(tgt).cuda()
    d = img - t
    loss = float(d.abs().mean())
    dimg = (torch.sign(d) / d.numel()).contiguous()
    gr = raster.render_backward(f, dg, dimg)
    return img.cpu().numpy(), loss, {k: gr[k].cpu().numpy() for k in PARAMS}


@pytest.mark.parametrize("persistent,use_graph", [(True, True), (False, False), (True, False)])
def test_batch_matches_plain_path_per_cell(persistent, use_graph):
    _case(f"batch persistent={persistent} graph={use_graph}")
    cells = _cells()
    ref = [_plain(g, cam, tgt, (16, 16)) for g, cam, tgt in cells]
    dgs = [raster.DeviceGaussians.from_host(g) for g, _, _ in cells]
    b = BatchStep(dgs, [c for _, c, _ in cells], [torch.as_tensor(t).cuda() for _, _, t in cells],
                  persistent=persistent, use_graph=use_graph)
    b.step()
    torch.cuda.synchronize()
    st, pairs = b.status()
    assert st == 0
    loss = b.loss.cpu().numpy()
    for c, (img, l1, gr) in enumerate(ref):
        np.testing.assert_array_equal(b.image(c).cpu().numpy(), img, err_msg=f"cell {c}")
        assert abs(loss[c] - l1) <= 1e-6 * max(l1, 1e-6) + 1e-7, (c, loss[c], l1)
        got = b.cell_grads(c)
        for k in PARAMS:
            grad_close(f"cell {c} {k}", got[k].cpu().numpy(), gr[k])
    b.close()


def test_batch_graph_replays_repeat_the_result():
    _case("graph replays")
    cells = _cells()
    dgs = [raster.DeviceGaussians.from_host(g) for g, _, _ in cells]
    b = BatchStep(dgs, [c for _, c, _ in cells], [torch.as_tensor(t).cuda() for _, _, t in cells])
    assert b.info()["use_graph"]
    b.step()
    torch.cuda.synchronize()
    img0 = b.images.cpu().numpy().copy()
    g0 = [{k: v.cpu().numpy().copy() for k, v in b.cell_grads(c).items()} for c in range(len(cells))]
    scratch = torch.randn(1 << 20, device="cuda")
    for rep in range(3):
        scratch.mul_(1.0001).add_(1.0)      # eager work between replays
        torch.cuda.synchronize()
        b.step()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(b.images.cpu().numpy(), img0, err_msg=f"replay {rep}")
        for c in range(len(cells)):
            got = b.cell_grads(c)
            for k in PARAMS:
                grad_close(f"replay {rep} cell {c} {k}", got[k].cpu().numpy(), g0[c][k])
    b.close()


def test_batch_autotune_picks_a_timed_candidate_and_stays_exact():
    _case("autotune")
    cells = _cells()
    dgs = [raster.DeviceGaussians.from_host(g) for g, _, _ in cells]
    b = BatchStep(dgs, [c for _, c, _ in cells], [torch.as_tensor(t).cuda() for _, _, t in cells], autotune=True)
    info = b.info()
    timed = [c for c in info["candidates"] if c["ms"] > 0]
    assert len(timed) == len(info["candidates"]) == 10
    # the search covers tile shapes, both launch forms, both LDS sizes and two grid sizes
    assert {c["fwd_batch"] for c in timed} == {128, 256} and {c["item_cap"] for c in timed} == {256, 512}
    assert {c["grid_pct"] for c in timed} == {75, 100} and {c["persistent"] for c in timed} == {True, False}
    best = min(timed, key=lambda c: c["ms"])
    assert tuple(best["tile"]) == tuple(info["tile"]) and best["persistent"] == info["persistent"]
    assert (best["fwd_batch"], best["item_cap"], best["grid_pct"]) == \
        (info["fwd_batch"], info["item_cap"], info["grid_pct"])
    print("autotune:", info)
    b.step()
    torch.cuda.synchronize()
    g, cam, _ = cells[0]
    ref = oracle.render(g, cam)
    image_close("autotuned cell 0", b.image(0).cpu().numpy(), ref["image"], ref["flags"])
    b.close()


@pytest.mark.parametrize("tile", [(16, 16), (32, 32)])
def test_batch_lds_knobs_and_grid_share_leave_every_bit_unchanged(tile):
    """The forward's LDS batch (128 or 256 entries), the backward's slot
    capacity (256 or 512) and the persistent grid's share change where the
    work is cut, not the order of any pixel's or entry's arithmetic: images
    and gradients are bitwise those of the default configuration, and the
    images those of the plain path."""
    _case(f"lds knobs tile={tile}")
    cells = _cells()
    dgs = [raster.DeviceGaussians.from_host(g) for g, _, _ in cells]
    cams, tgts = [c for _, c, _ in cells], [torch.as_tensor(t).cuda() for _, _, t in cells]
    ref = [_plain(g, cam, tgt, tile)[0] for g, cam, tgt in cells]

    def run(**kw):
        b = BatchStep(dgs, cams, tgts, tile=tile, **kw)
        b.step()
        torch.cuda.synchronize()
        assert b.status()[0] == 0
        out = (b.images.cpu().numpy().copy(),
               [{k: v.cpu().numpy().copy() for k, v in b.cell_grads(c).items()} for c in range(len(cells))],
               b.info())
        b.close()
        return out

    img0, g0, _ = run()
    img1, g1, info = run(fwd_batch=128, item_cap=256, grid_pct=60)
    assert (info["fwd_batch"], info["item_cap"], info["grid_pct"]) == (128, 256, 60)
    np.testing.assert_array_equal(img1, img0)
    for c in range(len(cells)):
        for k in PARAMS:
            np.testing.assert_array_equal(g1[c][k], g0[c][k], err_msg=f"cell {c} {k}")
    off = 0
    for c, (h, w) in enumerate([(cam.height, cam.width) for cam in cams]):
        np.testing.assert_array_equal(img1[off:off + 3 * h * w].reshape(3, h, w), ref[c], err_msg=f"cell {c}")
        off += 3 * h * w


def test_batch_rejects_unsupported_lds_knobs():
    cells = _cells()[:1]
    dgs = [raster.DeviceGaussians.from_host(g) for g, _, _ in cells]
    from paper_2402_17427_amd import _native as N
    for kw in (dict(fwd_batch=64), dict(item_cap=100), dict(grid_pct=101)):
        with pytest.raises(N.GsError):
            BatchStep(dgs, [c for _, c, _ in cells], [torch.as_tensor(t).cuda() for _, _, t in cells], **kw)


def _raw_planes(opt):
    dg = opt.dg
    return np.concatenate([dg.mean.cpu().numpy(), opt.log_scale.cpu().numpy(), dg.quat.cpu().numpy(),
                           opt.logit_opacity.cpu().numpy()[None], dg.sh.cpu().numpy()], axis=0)


def test_batch_training_step_with_eq1_loss_and_optimiser():
    """A complete training step of every cell in one graph replay: Eq. 1
    loss (lambda 0.2), backward, Adam with the densification statistics.
    Per cell and step: the image and loss equal the plain path's
    (single-view calls, gs_loss) bit for bit, the gradients are within
    tolerance of the plain path's, and the optimiser's result is the FP64
    oracle's Adam step from the pre-step state with the batch's own
    gradients and the step number the device schedule reached (1, then 2)."""
    from paper_2402_17427_amd import loss as gl
    from paper_2402_17427_amd import optim
    from gpu_util import adam_close
    _case("batch training step")
    cells = _cells()
    hyper = dict(optim.DEFAULTS, lr_mean=1e-3)
    dgs = [raster.DeviceGaussians.from_host(g) for g, _, _ in cells]
    opts = [optim.Adam.from_activated(dg) for dg in dgs]
    tg = [torch.as_tensor(t).cuda() for _, _, t in cells]
    b = BatchStep(dgs, [c for _, c, _ in cells], tg, loss_lambda=0.2, optimizers=opts, **hyper)
    assert b.info()["use_graph"]
    # plain path on separate copies
    pdgs = [raster.DeviceGaussians.from_host(g) for g, _, _ in cells]
    popts = [optim.Adam.from_activated(dg) for dg in pdgs]
    frames = []
    for dg, (_, cam, _) in zip(pdgs, cells):
        f = raster.Frame(dg.n, dg.sh_degree, cam)
        f.ensure_capacity(dg)
        frames.append(f)
    losses = [gl.ImageLoss(3, c.height, c.width) for _, c, _ in cells]
    deg = cells[0][0].sh_degree
    for step in (1, 2):
        pre = [(_raw_planes(o), o.m.cpu().numpy(), o.v.cpu().numpy()) for o in opts]
        b.step()
        torch.cuda.synchronize()
        assert b.status()[0] == 0
        for c, (f, dg, o, L) in enumerate(zip(frames, pdgs, popts, losses)):
            f.project(dg)
            f.bin_sort()
            f.render_fwd()
            lv, dimg, _ = L(f.image, tg[c], 0.2)
            f.render_bwd(dg, dimg)
            img_p = f.image.cpu().numpy()
            gr_p = f.grads()
            o.step(f, **hyper)
            torch.cuda.synchronize()
            if step == 1:
                # same parameters before the first step: same image and loss
                np.testing.assert_array_equal(b.image(c).cpu().numpy(), img_p, err_msg=f"cell {c}")
                assert float(b.loss[c]) == float(lv[0]), (c, float(b.loss[c]), float(lv[0]))
                got = b.cell_grads(c)
                for k in PARAMS:
                    grad_close(f"cell {c} {k}", got[k].cpu().numpy(), gr_p[k].cpu().numpy())
                np.testing.assert_array_equal(opts[c].visible_count.cpu().numpy()[:dg.n],
                                              o.visible_count.cpu().numpy()[:dg.n])
            # the batch's optimiser against the oracle from its own state
            n = dgs[c].n
            gb = b.cell_grads(c)
            ga = np.concatenate([gb["mean"].cpu().numpy(), gb["scale"].cpu().numpy(), gb["quat"].cpu().numpy(),
                                 gb["opacity"].cpu().numpy()[None], gb["sh"].cpu().numpy()], axis=0)
            raw0, m0, v0 = pre[c]
            got = dict(raw=_raw_planes(opts[c])[:, :n], m=opts[c].m.cpu().numpy()[:, :n],
                       v=opts[c].v.cpu().numpy()[:, :n], scale=dgs[c].scale.cpu().numpy()[:, :n],
                       opacity=dgs[c].opacity.cpu().numpy()[:n])
            adam_close(raw0[:, :n], m0[:, :n], v0[:, :n], ga[:, :n], got, hyper, deg, step)
    b.close()


def test_batch_above_the_onesweep_grid_matches_plain_path():
    """Three large cells (1.6M, 2.0M and 2.5M Gaussians, one 1600x1066 view
    each) sort more than 2048 x 4096 pairs jointly, so the onesweep passes
    take their partitions from the atomic counter.  Per cell the image is
    bit-identical to the plain path's and the gradients are within
    tolerance of it."""
    _case("batch above the onesweep grid")
    cells = []
    for i, (g, cam) in enumerate(scenes.config4(sizes=(1_600_000, 2_000_000, 2_500_000))):
        tgt = np.random.default_rng(700 + i).uniform(0, 1, (3, cam.height, cam.width)).astype(np.float32)
        cells.append((g, cam, tgt))
    ref = [_plain(g, cam, tgt, (16, 16)) for g, cam, tgt in cells]
    torch.cuda.empty_cache()
    dgs = [raster.DeviceGaussians.from_host(g) for g, _, _ in cells]
    b = BatchStep(dgs, [c for _, c, _ in cells], [torch.as_tensor(t).cuda() for _, _, t in cells],
                  persistent=False, use_graph=False)
    b.step()
    torch.cuda.synchronize()
    st, pairs = b.status()
    print(f"[case] {pairs} pairs", flush=True)
    assert st == 0 and pairs[0] > 2048 * 4096
    loss = b.loss.cpu().numpy()
    for c, (img, l1, gr) in enumerate(ref):
        np.testing.assert_array_equal(b.image(c).cpu().numpy(), img, err_msg=f"cell {c}")
        assert abs(loss[c] - l1) <= 1e-6 * max(l1, 1e-6) + 1e-7, (c, loss[c], l1)
        got = b.cell_grads(c)
        for k in PARAMS:
            grad_close(f"cell {c} {k}", got[k].cpu().numpy(), gr[k])
    b.close()
