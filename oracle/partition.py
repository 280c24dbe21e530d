"""Plain CPU oracle for the progressive data partitioning -- TEST INFRASTRUCTURE.

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's `cpu_baseline`
leg may import this module; the library's partitioning shares nothing with
it.

What it computes (VastGaussian, arXiv 2402.17427, section 4.1, and the
merging of section 4.3), in float64, step by step:
  1. camera-position-based region division: camera centres projected on
     the ground plane (world y is up; the ground coordinates are (x, z)),
     split into m sections along x with |V|/m views each, each section into
     n segments along z with |V|/(m n) views each;
  2. position-based data selection: each region's rectangle expanded by a
     ratio (0.2) of its side lengths, views and points whose ground
     position lies in the expanded rectangle assigned to the cell;
  3. visibility-based camera selection: for every camera not yet in the
     cell, the airspace-aware visibility = area of the image covered by the
     projection of the cell's box (the axis-aligned box of the cell's
     points, from the ground plane up to their highest point) over the
     image area; cameras above the threshold (0.25) join the cell;
  4. coverage-based point selection: points seen by any view of the cell
     (in front of the near plane, projecting inside the image) join it;
  5. merging: after optimisation a cell keeps only the Gaussians inside its
     original (unexpanded) rectangle.
Readings where the paper is silent: the sections' counts follow
numpy.array_split (the first |V| mod m sections take one view more),
boundaries lie midway between the neighbouring camera positions, the
outermost boundaries are the bounding rectangle of all camera positions and
points; the expansion keeps the rectangle's centre; the expanded
rectangles (which overlap) are closed, the original ones (which tile the
scene) half-open [lo, hi) except at the outermost upper edges;
the cell's box is formed by the points selected by position (step 2);
the box's part behind the near plane is clipped off before projecting;
"covered by the views" is the union of the views' frusta, occlusion
ignored.
"""
from __future__ import annotations

import numpy as np

EXPAND = 0.2
VISIBILITY = 0.25


def camera_centre(cam) -> np.ndarray:
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64).reshape(3)
    return -R.T @ t


def split_counts(count: int, parts: int):
    """Sizes of numpy.array_split(range(count), parts)."""
    return [len(a) for a in np.array_split(np.arange(count), parts)]


def _boundaries(sorted_vals, counts, lo, hi):
    """Edges of consecutive groups of sorted values: midpoints between the
    last value of a group and the first of the next; lo/hi outside."""
    edges = [lo]
    k = 0
    for c in counts[:-1]:
        k += c
        if k <= 0 or k >= len(sorted_vals):
            edges.append(edges[-1])
        else:
            edges.append(0.5 * (sorted_vals[k - 1] + sorted_vals[k]))
    edges.append(hi)
    return edges


def region_division(centres: np.ndarray, points: np.ndarray, m: int, n: int) -> np.ndarray:
    """[m*n][4] rectangles (x0, x1, z0, z1), cell index = i * n + j."""
    c = np.asarray(centres, np.float64)
    p = np.asarray(points, np.float64).reshape(-1, 3)
    allx = np.concatenate([c[:, 0], p[:, 0]])
    allz = np.concatenate([c[:, 2], p[:, 2]])
    X0, X1, Z0, Z1 = allx.min(), allx.max(), allz.min(), allz.max()
    order = np.argsort(c[:, 0], kind="stable")
    xs = c[order, 0]
    xcounts = split_counts(len(c), m)
    xedges = _boundaries(xs, xcounts, X0, X1)
    out = np.zeros((m * n, 4))
    k = 0
    for i in range(m):
        members = order[k:k + xcounts[i]]
        k += xcounts[i]
        zs = np.sort(c[members, 2], kind="stable")
        zcounts = split_counts(len(members), n)
        zedges = _boundaries(zs, zcounts, Z0, Z1)
        for j in range(n):
            out[i * n + j] = (xedges[i], xedges[i + 1], zedges[j], zedges[j + 1])
    return out


def expand(rect, ratio=EXPAND):
    x0, x1, z0, z1 = rect
    hx, hz = 0.5 * ratio * (x1 - x0), 0.5 * ratio * (z1 - z0)
    return (x0 - hx, x1 + hx, z0 - hz, z1 + hz)


def inside(x, z, rect, closed_hi=(False, False)):
    """x, z in the rectangle [x0, x1) x [z0, z1) (closed where asked)."""
    x0, x1, z0, z1 = rect
    okx = (x >= x0) & ((x <= x1) if closed_hi[0] else (x < x1))
    okz = (z >= z0) & ((z <= z1) if closed_hi[1] else (z < z1))
    return okx & okz


def cell_box(points_sel: np.ndarray):
    """Airspace box (x0, y0, z0, x1, y1, z1): the points' x, z extents, y
    from the ground (0) to the highest point."""
    if len(points_sel) == 0:
        return None
    lo = points_sel.min(axis=0)
    hi = points_sel.max(axis=0)
    return (lo[0], 0.0, lo[2], hi[0], max(hi[1], 0.0), hi[2])


def _box_corners(b):
    x0, y0, z0, x1, y1, z1 = b
    return np.array([[x, y, z] for x in (x0, x1) for y in (y0, y1) for z in (z0, z1)], np.float64)


_EDGES = [(a, b) for a in range(8) for b in range(a + 1, 8) if bin(a ^ b).count("1") == 1]


def _hull(pts):
    """Convex hull (Andrew's monotone chain), counter-clockwise."""
    pts = sorted(set(map(tuple, pts)))
    if len(pts) < 3:
        return pts

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return lower[:-1] + upper[:-1]


def _clip(poly, axis, value, keep_greater):
    """Sutherland-Hodgman against one axis-aligned line."""
    out = []
    n = len(poly)
    for k in range(n):
        a, b = poly[k], poly[(k + 1) % n]
        ina = a[axis] >= value if keep_greater else a[axis] <= value
        inb = b[axis] >= value if keep_greater else b[axis] <= value
        if ina:
            out.append(a)
        if ina != inb:
            t = (value - a[axis]) / (b[axis] - a[axis])
            out.append((a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1])))
    return out


def _area(poly):
    if len(poly) < 3:
        return 0.0
    s = 0.0
    for k in range(len(poly)):
        a, b = poly[k], poly[(k + 1) % len(poly)]
        s += a[0] * b[1] - b[0] * a[1]
    return abs(s) * 0.5


def visibility(cam, box) -> float:
    """Airspace-aware visibility of a box in a camera: the image area
    covered by the projection of the box's part in front of the near plane,
    over the image area."""
    if box is None:
        return 0.0
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64).reshape(3)
    cw = (R @ _box_corners(box).T).T + t
    near = float(cam.near)
    verts = [v for v in cw if v[2] > near]
    for a, b in _EDGES:
        za, zb = cw[a][2] - near, cw[b][2] - near
        if (za > 0) != (zb > 0):
            s = za / (za - zb)
            verts.append(cw[a] + s * (cw[b] - cw[a]))
    if len(verts) < 3:
        return 0.0
    uv = [(cam.fx * v[0] / v[2] + cam.cx, cam.fy * v[1] / v[2] + cam.cy) for v in verts]
    poly = _hull(uv)
    W, H = float(cam.width), float(cam.height)
    for axis, value, keep in ((0, 0.0, True), (0, W, False), (1, 0.0, True), (1, H, False)):
        if len(poly) < 3:
            return 0.0
        poly = _clip(poly, axis, value, keep)
    return _area(poly) / (W * H)


def covered(cam, pts: np.ndarray) -> np.ndarray:
    """Points in front of the near plane whose projection is in the image."""
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float64).reshape(3)
    q = pts @ R.T + t
    z = q[:, 2]
    front = z > cam.near
    zz = np.where(front, z, 1.0)
    u = cam.fx * q[:, 0] / zz + cam.cx
    v = cam.fy * q[:, 1] / zz + cam.cy
    return front & (u >= 0) & (u < cam.width) & (v >= 0) & (v < cam.height)


def partition(cams, points, m, n, ratio=EXPAND, threshold=VISIBILITY):
    """Steps 1-4.  Returns dict bounds [m*n][4], expanded [m*n][4],
    boxes (list), visibility [m*n][V], view_member [m*n][V] (0 / 1 by
    position / 2 by visibility), point_member [m*n][P] (0 / 1 by position /
    2 by coverage)."""
    pts = np.asarray(points, np.float64).reshape(-1, 3)
    centres = np.array([camera_centre(c) for c in cams])
    bounds = region_division(centres, pts, m, n)
    ncell, nv = m * n, len(cams)
    exp = np.array([expand(b, ratio) for b in bounds])
    vm = np.zeros((ncell, nv), np.uint8)
    pm = np.zeros((ncell, len(pts)), np.uint8)
    vis = np.zeros((ncell, nv))
    boxes = []
    for j in range(ncell):
        vm[j, inside(centres[:, 0], centres[:, 2], exp[j], (True, True))] = 1
        sel = inside(pts[:, 0], pts[:, 2], exp[j], (True, True))
        pm[j, sel] = 1
        box = cell_box(pts[sel])
        boxes.append(box)
        for i in range(nv):
            if vm[j, i] == 0:
                vis[j, i] = visibility(cams[i], box)
                if vis[j, i] > threshold:
                    vm[j, i] = 2
        for i in np.nonzero(vm[j])[0]:
            cov = covered(cams[i], pts) & (pm[j] == 0)
            pm[j, cov] = 2
    return dict(bounds=bounds, expanded=exp, boxes=boxes, visibility=vis, view_member=vm, point_member=pm)


def merge_keep(means_xz, rect, closed_hi=(False, False)):
    """Section 4.3: a cell keeps the Gaussians inside its original rectangle."""
    x, z = np.asarray(means_xz[0], np.float64), np.asarray(means_xz[1], np.float64)
    return inside(x, z, rect, closed_hi)
