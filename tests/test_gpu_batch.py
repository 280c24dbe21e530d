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
    assert len(timed) == len(info["candidates"]) >= 4
    best = min(timed, key=lambda c: c["ms"])
    assert tuple(best["tile"]) == tuple(info["tile"]) and best["persistent"] == info["persistent"]
    print("autotune:", info)
    b.step()
    torch.cuda.synchronize()
    g, cam, _ = cells[0]
    ref = oracle.render(g, cam)
    image_close("autotuned cell 0", b.image(0).cpu().numpy(), ref["image"], ref["flags"])
    b.close()
