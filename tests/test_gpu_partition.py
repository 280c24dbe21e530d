"""GPU parity of the point selection and merge mask of the partitioning
(VastGaussian, arXiv 2402.17427, sections 4.1 and 4.3) against the
partitioning oracle.

The kernel gets the view-side result of the library's host call; the oracle
is given the same expanded rectangles and view memberships, so the
position decisions (FP32 points against FP64 rectangles) are compared bit
for bit.  The coverage test is FP64 on both sides but the kernel
multiplies where the oracle divides, so a point is flagged when its
projection lies within 1e-6 px of an image edge or its depth within 1e-9 m
of the near plane in some view of the cell; memberships must be identical
at every unflagged point, and flagged points must be rare.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gen import scenes
from oracle import partition as P
from paper_2402_17427_amd import partition as gp

pytestmark = pytest.mark.gpu


def _case(name):
    print(f"\n[case] {name}", flush=True)


def _oracle_members(cams, pts, expanded, vm):
    """Oracle selection with the library's rectangles and view sets, plus
    the ambiguity flags."""
    nc = len(expanded)
    mem = np.zeros((nc, len(pts)), np.uint8)
    amb = np.zeros(len(pts), bool)
    for j in range(nc):
        ins = P.inside(pts[:, 0], pts[:, 2], expanded[j], (True, True))
        mem[j, ins] = 1
        for i in np.nonzero(vm[j])[0]:
            cam = cams[i]
            R = np.asarray(cam.R, np.float64).reshape(3, 3)
            q = pts @ R.T + np.asarray(cam.t, np.float64)
            z = q[:, 2]
            zz = np.where(z > 0, z, 1.0)
            u = cam.fx * q[:, 0] / zz + cam.cx
            v = cam.fy * q[:, 1] / zz + cam.cy
            near = np.abs(z - cam.near) < 1e-9
            edge = (z > cam.near) & (np.minimum.reduce([np.abs(u), np.abs(u - cam.width), np.abs(v),
                                                         np.abs(v - cam.height)]) < 1e-6)
            amb |= (near | edge) & ~ins
            cov = P.covered(cam, pts) & (mem[j] == 0)
            mem[j, cov] = 2
    return mem, amb


@pytest.mark.parametrize("seed,V,Pn,m,n", [(1, 60, 20000, 2, 2), (2, 150, 50000, 2, 4), (3, 9, 1, 3, 1),
                                           (4, 40, 4099, 1, 1)])
def test_select_points_matches_the_oracle(seed, V, Pn, m, n):
    _case(f"select_points seed={seed} V={V} P={Pn} grid={m}x{n}")
    cams = scenes.aerial_survey(V, seed, extent_m=600.0, width=320, height=240)
    pts = scenes.sfm_points(Pn, seed + 1, extent_m=600.0)
    host = gp.partition_views(cams, pts, m, n)
    sel = gp.PointSelector(V, m * n, Pn)
    dev = torch.as_tensor(np.ascontiguousarray(pts.T)).cuda()
    tests = torch.zeros(1, dtype=torch.int64, device="cuda")
    got = sel(dev, cams, host["expanded"], host["view_member"], tests=tests)
    torch.cuda.synchronize()
    got = got.cpu().numpy()[:, :Pn]
    ref, amb = _oracle_members(cams, pts.astype(np.float64), host["expanded"], host["view_member"])
    assert amb.mean() < 1e-3
    np.testing.assert_array_equal(got[:, ~amb], ref[:, ~amb])
    # projections run only for points outside a cell's expanded rectangle
    assert (int(tests.item()) > 0) == bool((ref != 1).any())


def test_full_survey_sampled_points():
    """The benchmark's survey (1000 views at 1152x864 over 1 km^2, 2M
    points, 2 x 4 cells) in the launch the benchmark times; the oracle
    checks a random sample of 20k points (each point's membership depends
    on that point only)."""
    _case("select_points survey 1000 views x 2M points")
    cams = scenes.aerial_survey(1000, 7)
    pts = scenes.sfm_points(2_000_000, 8)
    host = gp.partition_views(cams, pts, 2, 4)
    sel = gp.PointSelector(len(cams), 8, len(pts))
    dev = torch.as_tensor(np.ascontiguousarray(pts.T)).cuda()
    got = sel(dev, cams, host["expanded"], host["view_member"])
    torch.cuda.synchronize()
    idx = np.random.default_rng(9).choice(len(pts), 20000, replace=False)
    sub = pts[idx].astype(np.float64)
    ref, amb = _oracle_members(cams, sub, host["expanded"], host["view_member"])
    g = got.cpu().numpy()[:, idx]
    assert amb.mean() < 1e-3
    np.testing.assert_array_equal(g[:, ~amb], ref[:, ~amb])
    assert (g == 2).any() and (g == 1).any()


def test_merge_keep_matches_the_oracle_and_partitions_the_points():
    _case("merge_keep")
    cams = scenes.aerial_survey(80, 11, extent_m=600.0, width=320, height=240)
    pts = scenes.sfm_points(30001, 12, extent_m=600.0)
    host = gp.partition_views(cams, pts, 2, 3)
    b = host["bounds"]
    X1, Z1 = b[:, 1].max(), b[:, 3].max()
    dev = torch.as_tensor(np.ascontiguousarray(pts.T)).cuda()
    keeps = []
    for j in range(6):
        closed = (b[j, 1] == X1, b[j, 3] == Z1)
        k = gp.merge_keep(dev, b[j], closed).cpu().numpy()
        ref = P.merge_keep((pts[:, 0].astype(np.float64), pts[:, 2].astype(np.float64)), b[j], closed)
        np.testing.assert_array_equal(k.astype(bool), ref)
        keeps.append(k)
    np.testing.assert_array_equal(np.sum(keeps, axis=0), 1)
