"""Central finite differences of the FP64 oracle's forward for a few
Gaussians of a large scene.  A perturbation of Gaussian i changes only the
pixels its support reaches, so each difference re-renders only those
pixels (its pixel rectangle plus a margin) with the Gaussians whose
support meets them; every other Gaussian has alpha < 1/255 there."""
from __future__ import annotations

import numpy as np

import oracle
from gen import scenes

PARAMS = ("mean", "scale", "quat", "opacity", "sh")


def support_rect(pxrect, W, H, margin=2):
    x0, y0, x1, y1 = pxrect
    return max(x0 - margin, 0), max(y0 - margin, 0), min(x1 + margin, W - 1), min(y1 + margin, H - 1)


def pick_gaussians(g, cam, count, seed, max_area=300):
    pr = oracle.project(g, cam)
    valid = pr["valid"] != 0
    rect = pr["pxrect"].astype(np.int64)
    area = (rect[:, 2] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 1] + 1)
    rng = np.random.default_rng(seed)
    cand = np.nonzero(valid & (area <= max_area) & (area >= 4))[0]
    pick = np.sort(rng.choice(cand, count, replace=False))
    return pick, valid, rect


def loss_weights(g, cam, pick, rect, seed):
    """Seeded w ~ N(0, 1) on the pixels around the picked Gaussians, 0 at
    pixels the oracle flags as ambiguous and everywhere else."""
    W, H = cam.width, cam.height
    mask = np.zeros((H, W), bool)
    for i in pick:
        x0, y0, x1, y1 = support_rect(rect[i], W, H)
        mask[y0:y1 + 1, x0:x1 + 1] = True
    py, px = np.nonzero(mask)
    fl = oracle.render(g, cam, px.astype(np.int32), py.astype(np.int32))["flags"]
    rng = np.random.default_rng(seed)
    wv = rng.standard_normal((3, px.size)).astype(np.float32)
    wv[:, fl != 0] = 0.0
    w = np.zeros((3, H, W), np.float32)
    w[:, py, px] = wv
    return w


def central_differences(g, cam, pick, valid, rect, w, h=1e-4):
    """dL/dtheta by central differences for every parameter of each picked
    Gaussian, L = sum(w * I).  Returns {param: [(gaussian, row, value)]} and
    the number of components skipped because a +-h evaluation put a
    weighted pixel within a threshold's window."""
    W, H = cam.width, cam.height
    out = {k: [] for k in PARAMS}
    skipped = 0
    for i in pick:
        x0, y0, x1, y1 = support_rect(rect[i], W, H)
        near = valid & (rect[:, 0] <= x1) & (rect[:, 2] >= x0) & (rect[:, 1] <= y1) & (rect[:, 3] >= y0)
        near[i] = True
        idx = np.nonzero(near)[0]
        j = int(np.nonzero(idx == i)[0][0])
        ys, xs = np.mgrid[y0:y1 + 1, x0:x1 + 1]
        qx, qy = xs.ravel().astype(np.int32), ys.ravel().astype(np.int32)
        wq = w[:, qy, qx].astype(np.float64)
        live = np.abs(wq).sum(0) > 0
        sub = g.subset(idx)
        sub = scenes.Gaussians(*(np.array(getattr(sub, k), np.float64) for k in PARAMS), g.sh_degree)
        for k in PARAMS:
            arr = getattr(sub, k)
            view = arr if arr.ndim == 2 else arr[None, :]
            for r in range(view.shape[0]):
                vals, ok, dec = [], True, []
                for sgn in (1.0, -1.0):
                    view[r, j] += sgn * h
                    o = oracle.render(sub, cam, qx, qy)
                    view[r, j] -= sgn * h
                    ok &= not (o["flags"][live] != 0).any()
                    vals.append(float((o["image"].T * wq).sum()))
                    dec.append((o["nblend"][live], o["last_id"][live]))
                # a decision (alpha vs 1/255, the stop) that differs between
                # the two evaluations makes the difference meaningless
                ok &= bool((dec[0][0] == dec[1][0]).all() and (dec[0][1] == dec[1][1]).all())
                if ok:
                    out[k].append((int(i), r, (vals[0] - vals[1]) / (2 * h)))
                else:
                    skipped += 1
    return out, skipped


def gather(grads, fd):
    """Pick the analytic values matching the finite differences."""
    got, want = {}, {}
    for k, items in fd.items():
        a = np.asarray(grads[k], np.float64)
        a = a if a.ndim == 2 else a[None, :]
        got[k] = np.array([a[r, i] for i, r, _ in items])
        want[k] = np.array([v for _, _, v in items])
    return got, want
