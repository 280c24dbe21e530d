"""Pins of the partitioning oracle (VastGaussian, arXiv 2402.17427, section
4.1 progressive data partitioning, section 4.3 merging).

The oracle is checked against what the method fixes independently of its
code: balanced view counts per section and segment, regions that tile the
scene without overlap, the 1.2x expansion about the centre, the visible
area of a box from brute-force ray casting of every pixel, closed cases
(a box filling the view, a box behind the camera), the polygon primitives
on known shapes, and the invariants every selection must satisfy.
"""
import math

import numpy as np
import pytest

from gen import scenes
from oracle import partition as P


def _cam_at(pos, target, w=160, h=120, hfov=60.0):
    return scenes.look_at(np.asarray(pos, np.float64), np.asarray(target, np.float64), w, h, hfov_deg=hfov)


def _survey(seed, n_views=120, extent=400.0, w=160, h=120):
    rng = np.random.default_rng(seed)
    cams = []
    for _ in range(n_views):
        x, z = rng.uniform(-extent / 2, extent / 2, 2)
        alt = rng.uniform(80, 160)
        yaw = rng.uniform(0, 2 * math.pi)
        d = rng.uniform(20, 120)
        tgt = (x + d * math.cos(yaw), 0.0, z + d * math.sin(yaw))
        cams.append(_cam_at((x, alt, z), tgt, w, h))
    pts = np.stack([rng.uniform(-extent / 2, extent / 2, 3000), rng.uniform(0, 40, 3000),
                    rng.uniform(-extent / 2, extent / 2, 3000)], axis=1)
    return cams, pts


def test_region_division_balances_views_and_tiles_the_scene():
    cams, pts = _survey(1, n_views=121)
    m, n = 3, 4
    c = np.array([P.camera_centre(k) for k in cams])
    b = P.region_division(c, pts, m, n)
    X0, X1 = min(c[:, 0].min(), pts[:, 0].min()), max(c[:, 0].max(), pts[:, 0].max())
    Z0, Z1 = min(c[:, 2].min(), pts[:, 2].min()), max(c[:, 2].max(), pts[:, 2].max())
    # tiling: areas add up to the extent, no two overlap
    area = ((b[:, 1] - b[:, 0]) * (b[:, 3] - b[:, 2])).sum()
    assert abs(area - (X1 - X0) * (Z1 - Z0)) < 1e-6 * area
    for i in range(len(b)):
        for j in range(i + 1, len(b)):
            ox = min(b[i, 1], b[j, 1]) - max(b[i, 0], b[j, 0])
            oz = min(b[i, 3], b[j, 3]) - max(b[i, 2], b[j, 2])
            assert ox <= 0 or oz <= 0
    # every camera in exactly one region; counts as balanced as possible
    cnt = np.zeros(len(b), int)
    for k in range(len(c)):
        hits = [j for j in range(len(b)) if P.inside(c[k, 0], c[k, 2], b[j], (b[j, 1] == X1, b[j, 3] == Z1))]
        assert len(hits) == 1, k
        cnt[hits[0]] += 1
    sec = cnt.reshape(m, n).sum(axis=1)
    assert sec.max() - sec.min() <= 1 and sec.sum() == len(c)
    for i in range(m):
        assert cnt.reshape(m, n)[i].max() - cnt.reshape(m, n)[i].min() <= 1


def test_expansion_is_twenty_percent_about_the_centre():
    r = (10.0, 30.0, -5.0, 35.0)
    e = P.expand(r)
    assert abs((e[1] - e[0]) - 1.2 * 20.0) < 1e-12 and abs((e[3] - e[2]) - 1.2 * 40.0) < 1e-12
    assert abs((e[0] + e[1]) - (r[0] + r[1])) < 1e-12 and abs((e[2] + e[3]) - (r[2] + r[3])) < 1e-12


def _raycast_visibility(cam, box):
    """Fraction of pixel centres whose viewing ray meets the box beyond the
    near plane (slab test in world coordinates)."""
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    C = P.camera_centre(cam)
    ys, xs = np.meshgrid(np.arange(cam.height) + 0.5, np.arange(cam.width) + 0.5, indexing="ij")
    dc = np.stack([(xs - cam.cx) / cam.fx, (ys - cam.cy) / cam.fy, np.ones_like(xs)], axis=-1).reshape(-1, 3)
    d = dc @ R      # R^T applied to each row: world direction with camera z = 1 per unit s
    lo = np.array(box[:3])
    hi = np.array(box[3:])
    with np.errstate(divide="ignore", invalid="ignore"):
        t0 = (lo - C) / d
        t1 = (hi - C) / d
    tmin = np.nanmax(np.where(np.isfinite(np.minimum(t0, t1)), np.minimum(t0, t1), -np.inf), axis=1)
    tmax = np.nanmin(np.where(np.isfinite(np.maximum(t0, t1)), np.maximum(t0, t1), np.inf), axis=1)
    hit = tmax > np.maximum(tmin, cam.near)
    return hit.mean()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_visibility_matches_ray_casting(seed):
    rng = np.random.default_rng(seed)
    box = (-40.0, 0.0, -30.0, 50.0, rng.uniform(10, 60), 60.0)
    for _ in range(6):
        pos = (rng.uniform(-200, 200), rng.uniform(30, 200), rng.uniform(-200, 200))
        tgt = (rng.uniform(-60, 60), 0.0, rng.uniform(-60, 60))
        cam = _cam_at(pos, tgt, 200, 150)
        v = P.visibility(cam, box)
        rc = _raycast_visibility(cam, box)
        # pixel-centre sampling error: a band of about one pixel along the outline
        assert abs(v - rc) <= 0.012 + 0.02 * rc, (v, rc)


def test_visibility_closed_cases():
    box = (-1000.0, 0.0, -1000.0, 1000.0, 50.0, 1000.0)
    down = _cam_at((0.0, 100.0, 0.0), (0.0, 0.0, 1e-3), 64, 48)
    assert abs(P.visibility(down, box) - 1.0) < 1e-12
    # box entirely behind the camera
    cam = _cam_at((0.0, 10.0, 0.0), (0.0, 10.0, 100.0), 64, 48)
    assert P.visibility(cam, (-5.0, 0.0, -50.0, 5.0, 20.0, -20.0)) == 0.0
    # camera inside the box sees it everywhere
    assert abs(P.visibility(cam, (-50.0, 0.0, -50.0, 50.0, 50.0, 50.0)) - 1.0) < 1e-12
    assert P.visibility(cam, None) == 0.0


def test_polygon_primitives():
    h = P._hull([(0, 0), (2, 0), (2, 2), (0, 2), (1, 1), (1, 0)])
    assert abs(P._area(h) - 4.0) < 1e-15 and len(h) == 4
    sq = [(-1.0, -1.0), (3.0, -1.0), (3.0, 3.0), (-1.0, 3.0)]
    for axis, value, keep in ((0, 0.0, True), (0, 2.0, False), (1, 0.0, True), (1, 1.0, False)):
        sq = P._clip(sq, axis, value, keep)
    assert abs(P._area(sq) - 2.0) < 1e-15
    tri = [(0.0, 0.0), (4.0, 0.0), (0.0, 4.0)]
    assert abs(P._area(P._clip(tri, 0, 2.0, False)) - 6.0) < 1e-15


def test_coverage_of_single_points():
    cam = _cam_at((0.0, 0.0, 0.0), (0.0, 0.0, 10.0), 64, 48)
    pts = np.array([[0.0, 0.0, 10.0], [0.0, 0.0, -10.0], [1e3, 0.0, 10.0], [0.0, 0.0, 0.1]])
    np.testing.assert_array_equal(P.covered(cam, pts), [True, False, False, False])


def test_partition_invariants():
    cams, pts = _survey(5)
    out = P.partition(cams, pts, 2, 2)
    c = np.array([P.camera_centre(k) for k in cams])
    vm, pm = out["view_member"], out["point_member"]
    assert (vm.sum(axis=0) > 0).all()          # every view lands in some cell
    for j in range(4):
        e = out["expanded"][j]
        ins = P.inside(c[:, 0], c[:, 2], e, (True, True))
        assert np.all((vm[j] == 1) <= ins)
        assert np.all(out["visibility"][j][vm[j] == 2] > P.VISIBILITY)
        assert np.all(out["visibility"][j][vm[j] == 0] <= P.VISIBILITY)
        assert np.all((pm[j] == 1) == P.inside(pts[:, 0], pts[:, 2], e, (True, True)))
        cov = np.zeros(len(pts), bool)
        for i in np.nonzero(vm[j])[0]:
            cov |= P.covered(cams[i], pts)
        assert np.all((pm[j] == 2) == (cov & (pm[j] != 1)))


def test_merge_keeps_each_gaussian_once():
    cams, pts = _survey(6)
    c = np.array([P.camera_centre(k) for k in cams])
    b = P.region_division(c, pts, 2, 3)
    X1 = max(c[:, 0].max(), pts[:, 0].max())
    Z1 = max(c[:, 2].max(), pts[:, 2].max())
    keep = np.stack([P.merge_keep((pts[:, 0], pts[:, 2]), b[j], (b[j, 1] == X1, b[j, 3] == Z1))
                     for j in range(len(b))])
    np.testing.assert_array_equal(keep.sum(axis=0), 1)


def test_airspace_box_reaches_the_ground():
    pts = np.array([[1.0, 12.0, 3.0], [4.0, 30.0, -2.0], [2.0, 18.0, 7.0]])
    assert P.cell_box(pts) == (1.0, 0.0, -2.0, 4.0, 30.0, 7.0)


def test_planted_missing_near_clip_is_caught(monkeypatch):
    """Projecting every box corner, also those behind the camera, is a
    plausible slip; the closed case of a camera inside the box catches it
    (planted in the oracle, on the CPU)."""
    def no_clip(cam, box):
        R = np.asarray(cam.R, np.float64).reshape(3, 3)
        cw = (R @ P._box_corners(box).T).T + np.asarray(cam.t, np.float64)
        uv = [(cam.fx * v[0] / v[2] + cam.cx, cam.fy * v[1] / v[2] + cam.cy) for v in cw]
        poly = P._hull(uv)
        for axis, value, keep in ((0, 0.0, True), (0, float(cam.width), False), (1, 0.0, True),
                                  (1, float(cam.height), False)):
            if len(poly) < 3:
                return 0.0
            poly = P._clip(poly, axis, value, keep)
        return P._area(poly) / (cam.width * cam.height)

    monkeypatch.setattr(P, "visibility", no_clip)
    with pytest.raises(AssertionError):
        test_visibility_closed_cases()
