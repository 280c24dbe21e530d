#!/usr/bin/env python3
"""Throughput of the differentiable Gaussian tile rasterizer on one MI355X.

Workload: one partition cell of an aerial city reconstruction (VastGaussian,
arXiv 2402.17427, section 4.1 cells; section 3 renderer): 1,000,000
Gaussians with SH degree 3 on a 200 m x 200 m synthetic city heightfield,
one aerial view at 150 m altitude pitched -45 deg, 1920x1080, 16x16 tiles.
A step is one pass of the whole hot path: projection (EWA + SH), key
emission, onesweep radix sort, tile ranges, forward blend, backward blend
and the projection backward, with dL/dImage precomputed and every input
resident in HBM before timing.

Prints one JSON line: metric value in Mpix/s (W*H per fwd+bwd step),
the roofline of the dominant kernel (durations from HIP events recorded
around every stage over the timed steps), and the FP64 oracle timed on the
host on a bounded pixel sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts
HBM_PEAK_GBS = 8000.0
N_CU, LANES_PER_CU_CLK, CLOCK_GHZ = 256, 64, 2.4
VALU_PEAK_GOPS = N_CU * LANES_PER_CU_CLK * CLOCK_GHZ        # 39,321.6 G lane-ops/s (FP32, one op per lane per clock)

# Algorithmic VALU work per counted unit (lane-ops, transcendental = 4),
# minimal operation counts of the blend as defined in the method:
#  forward, per evaluation with alpha >= 1/255 up to the stop (support pair):
#    offsets 2 + quadratic form 5 + exp 4 + alpha 1 + cap 1 + tests 2
#    + transmittance 2 + stop test 1                                  = 18
#  forward, per blended pair: weight 1 + colour 3 fma + T/last update 2 = 6
#  backward, per blended pair: recompute (offsets 2, quadratic 5, exp 4,
#    alpha 2) 13 + T_i by division 5 + weight 1 + colour grads 3
#    + dalpha 9 + suffix colour 3 + opacity/power 2 + conic 6 + centre 6 = 48
FWD_OPS_SUPPORT = 18
FWD_OPS_BLEND = 6
BWD_OPS_BLEND = 48


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=32, help="oracle pixel sample: every n-th row and column")
    ap.add_argument("--tile", type=int, nargs=2, default=(16, 16))
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--width", type=int, default=1920)
    ap.add_argument("--height", type=int, default=1080)
    return ap.parse_args()


def cpu_baseline(g, cam, stride):
    """FP64 oracle fwd+bwd on a stratified pixel sample (every stride-th row
    and column), timed on the host; includes the oracle's per-view
    projection and depth sort."""
    import numpy as np
    import oracle
    from gen import scenes
    px, py = scenes.pixel_sample(cam.width, cam.height, stride=stride)
    rng = np.random.default_rng(2)
    dimg = np.zeros((3, cam.height, cam.width), np.float32)
    dimg[:, py, px] = rng.uniform(-1, 1, (3, px.size)).astype(np.float32)
    t0 = time.perf_counter()
    oracle.render(g, cam, px, py)
    oracle.backward(g, cam, dimg, px, py)
    dt = time.perf_counter() - t0
    return {"value": round(px.size / dt / 1e6, 6), "unit": "Mpix/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"fwd+bwd of {px.size} pixels (every {stride}th row and column of the {cam.width}x"
                      f"{cam.height} view, 1M Gaussians) in {dt:.1f} s, per-view projection and sort included"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures a single GPU; --gpus {args.gpus} is not supported (the rasterizer of one "
              f"partition cell runs on one GPU; cells shard one per GPU with no exchange)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from gen import scenes
    from paper_2402_17427_amd import _native as N
    from paper_2402_17427_amd import raster

    torch.cuda.set_device(0)
    g, cam = scenes.config2(n=args.n, width=args.width, height=args.height)
    dg = raster.DeviceGaussians.from_host(g)
    frame = raster.Frame(g.n, g.sh_degree, cam, tile=tuple(args.tile))
    P = frame.ensure_capacity(dg)
    dimg = torch.as_tensor(scenes.grad_image(cam, 2, "uniform")).cuda()

    def step():
        frame.project(dg)
        frame.bin_sort()
        frame.render_fwd()
        frame.render_bwd(dg, dimg)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    frame.check_status()
    print(f"[bench] warmup done, pairs={P}", file=sys.stderr, flush=True)

    N.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = N.profile_report()
    N.profile_enable(False)
    frame.check_status()
    ms = (t1 - t0) / args.steps * 1e3
    npix = cam.width * cam.height
    value = npix / (ms * 1e-3) / 1e6

    stats = frame.stats()
    stages = {k: round(v[0] / v[1], 4) for k, v in prof.items()}
    dom = max(prof, key=lambda k: prof[k][0])
    dom_ms = prof[dom][0] / prof[dom][1]
    if dom == "render_bwd":
        work = stats["blended"] * BWD_OPS_BLEND
    elif dom == "render_fwd":
        work = stats["support"] * FWD_OPS_SUPPORT + stats["blended"] * FWD_OPS_BLEND
    else:
        work = None
    roof = None
    if work is not None:
        achieved = work / (dom_ms * 1e-3) / 1e12     # T lane-ops/s
        peak = VALU_PEAK_GOPS / 1e3
        roof = {"bound": "alu", "kernel": dom, "achieved": round(achieved, 3), "peak": round(peak, 3),
                "unit": "Tlane-op/s", "frac": round(achieved / peak, 4), "traffic": None,
                "work_lane_ops": int(work), "avg_ms": round(dom_ms, 4)}

    out = {
        "metric": "fwd+bwd Mpix/s at 1M Gaussians 1080p",
        "value": round(value, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"one cell: {g.n} Gaussians SH3 on a 200 m city heightfield, aerial view "
                               f"{cam.width}x{cam.height} at 150 m / -45 deg, tiles {args.tile[0]}x{args.tile[1]}",
                   "gaussians": g.n, "width": cam.width, "height": cam.height, "pairs": P,
                   "blend_counts": stats, "stage_ms": stages},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, cam, args.cpu_stride)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
