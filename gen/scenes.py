"""Seeded synthetic scenes and cameras.

This module only draws inputs: Gaussian parameter sets, pinhole cameras,
loss-gradient images and request traces.  It holds none of the rasterizer's
arithmetic (no projection, no colour evaluation, no blending), so both the
FP64 oracle and the HIP path can consume its outputs without sharing code.

Layout of a Gaussian set (structure of arrays, float32, plane-major):
  mean    [3][N]    world position (x, y, z), world y-up
  scale   [3][N]    linear (already exponentiated) per-axis scale, > 0
  quat    [4][N]    rotation quaternion (w, x, y, z), any non-zero norm
  opacity [N]       activated opacity in (0, 1)
  sh      [3K][N]   spherical-harmonic coefficients, plane c*K + k for colour
                    channel c and basis index k = l*l + l + m, K = (deg+1)^2

Camera (float32 values): world->camera rotation R (row-major 3x3) and
translation t, camera +z forward, +x right, +y down; pinhole fx, fy, cx, cy;
image width/height; near plane; background colour.

The shapes and value distributions follow the aerial reconstruction setting
of VastGaussian (arXiv 2402.17427): 3D Gaussians with position, anisotropic
covariance, opacity and SH colour (section 3), scenes that are partitioned
into ground cells (section 4.1) and merged by concatenation (section 4.3).
Aerial datasets are not available, so a procedural city heightfield stands
in for the SfM-initialised Gaussians.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SH_DIM = {0: 1, 1: 4, 2: 9, 3: 16}


@dataclasses.dataclass
class Gaussians:
    mean: np.ndarray      # float32 [3][N]
    scale: np.ndarray     # float32 [3][N]
    quat: np.ndarray      # float32 [4][N]
    opacity: np.ndarray   # float32 [N]
    sh: np.ndarray        # float32 [3K][N]
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def subset(self, idx) -> "Gaussians":
        idx = np.asarray(idx)
        return Gaussians(np.ascontiguousarray(self.mean[:, idx]),
                         np.ascontiguousarray(self.scale[:, idx]),
                         np.ascontiguousarray(self.quat[:, idx]),
                         np.ascontiguousarray(self.opacity[idx]),
                         np.ascontiguousarray(self.sh[:, idx]),
                         self.sh_degree)

    def copy(self) -> "Gaussians":
        return Gaussians(self.mean.copy(), self.scale.copy(), self.quat.copy(),
                         self.opacity.copy(), self.sh.copy(), self.sh_degree)


@dataclasses.dataclass
class Camera:
    R: np.ndarray         # float32 [9] row-major world->camera rotation
    t: np.ndarray         # float32 [3]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)

    def as_f32(self) -> "Camera":
        f = lambda x: float(np.float32(x))
        return Camera(np.asarray(self.R, np.float32).reshape(9),
                      np.asarray(self.t, np.float32).reshape(3),
                      f(self.fx), f(self.fy), f(self.cx), f(self.cy),
                      int(self.width), int(self.height), f(self.near),
                      tuple(f(b) for b in self.bg))


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def look_at(eye, target, width, height, hfov_deg=60.0, near=0.2,
            bg=(0.0, 0.0, 0.0), world_up=(0.0, 1.0, 0.0)) -> Camera:
    """Pinhole camera at `eye` looking at `target`, world y-up, camera y-down."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    up = np.asarray(world_up, np.float64)
    r = np.cross(f, up)
    if np.linalg.norm(r) < 1e-9:          # looking straight down/up
        r = np.cross(f, np.array([0.0, 0.0, 1.0]))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)                    # camera +y points down in the image
    R = np.stack([r, d, f])               # rows: camera axes in world coords
    t = -R @ eye
    fx = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return Camera(R.reshape(9), t, fx, fx, width / 2.0, height / 2.0,
                  width, height, near, bg).as_f32()


def camera_from_pose(pos, yaw, pitch, width, height, hfov_deg=60.0, near=0.2,
                     bg=(0.0, 0.0, 0.0)) -> Camera:
    """Camera at `pos` with heading `yaw` (radians, about world y) and
    `pitch` (radians, negative looks down)."""
    d = np.array([math.cos(pitch) * math.sin(yaw), math.sin(pitch),
                  math.cos(pitch) * math.cos(yaw)])
    return look_at(pos, np.asarray(pos) + d, width, height, hfov_deg, near, bg)


# ---------------------------------------------------------------- city -----

def city_heightfield(rng, size_m, origin=(0.0, 0.0), block_m=25.0):
    """Axis-aligned block buildings on a flat ground, one per 25 m block.

    Returns (x0, z0, x1, z1, h) arrays describing building footprints."""
    nb = max(1, int(round(size_m / block_m)))
    ox = origin[0] - size_m / 2.0
    oz = origin[1] - size_m / 2.0
    bx, bz = np.meshgrid(np.arange(nb), np.arange(nb), indexing="ij")
    bx = bx.ravel()
    bz = bz.ravel()
    fw = rng.uniform(8.0, 18.0, bx.size)
    fd = rng.uniform(8.0, 18.0, bx.size)
    h = rng.uniform(5.0, 40.0, bx.size)
    offx = rng.uniform(0.0, 1.0, bx.size) * (block_m - fw)
    offz = rng.uniform(0.0, 1.0, bx.size) * (block_m - fd)
    x0 = ox + bx * block_m + offx
    z0 = oz + bz * block_m + offz
    return x0, z0, x0 + fw, z0 + fd, h, nb, ox, oz, block_m


def _height_at(x, z, hf):
    x0, z0, x1, z1, h, nb, ox, oz, block_m = hf
    i = np.clip(np.floor((x - ox) / block_m).astype(np.int64), 0, nb - 1)
    j = np.clip(np.floor((z - oz) / block_m).astype(np.int64), 0, nb - 1)
    b = i * nb + j
    inside = (x >= x0[b]) & (x < x1[b]) & (z >= z0[b]) & (z < z1[b])
    return np.where(inside, h[b], 0.0)


def city_gaussians(n, seed, size_m=200.0, origin=(0.0, 0.0), sh_degree=3,
                   log_scale=(-2.5, 0.7), opacity_logit_sd=1.5, jitter=0.5,
                   sh_rest_sd=0.05) -> Gaussians:
    """Gaussians with means on a synthetic city heightfield patch."""
    rng = np.random.default_rng(seed)
    hf = city_heightfield(rng, size_m, origin)
    x = rng.uniform(origin[0] - size_m / 2, origin[0] + size_m / 2, n)
    z = rng.uniform(origin[1] - size_m / 2, origin[1] + size_m / 2, n)
    y = _height_at(x, z, hf)
    mean = np.stack([x, y, z]) + rng.normal(0.0, jitter, (3, n))
    scale = np.exp(rng.normal(log_scale[0], log_scale[1], (3, n)))
    quat = _quats(rng, n)
    opacity = sigmoid(rng.normal(0.0, opacity_logit_sd, n))
    K = SH_DIM[sh_degree]
    sh = np.empty((3, K, n))
    sh[:, 0, :] = rng.uniform(0.0, 1.0, (3, n))
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, sh_rest_sd, (3, K - 1, n))
    return Gaussians(mean.astype(np.float32), scale.astype(np.float32),
                     quat.astype(np.float32), opacity.astype(np.float32),
                     sh.reshape(3 * K, n).astype(np.float32), sh_degree)


def aerial_camera(width, height, altitude, target=(0.0, 0.0, 0.0),
                  pitch_deg=-45.0, yaw=0.0, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Camera `altitude` metres above the target level, pitched down and
    looking at `target` along heading `yaw`."""
    p = math.radians(-pitch_deg)
    back = altitude / math.tan(p)
    tx, ty, tz = target
    eye = (tx - back * math.sin(yaw), ty + altitude, tz - back * math.cos(yaw))
    return look_at(eye, target, width, height, bg=bg)


# ------------------------------------------------------------- configs -----

def config1(seed=1):
    """2,000 Gaussians in a box in front of an identity camera, 128x128."""
    rng = np.random.default_rng(seed)
    n = 2000
    mean = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n),
                     rng.uniform(3, 6, n)])
    scale = np.exp(rng.normal(-3.0, 0.5, (3, n)))
    quat = _quats(rng, n)
    opacity = sigmoid(rng.normal(0.0, 1.0, n))
    rgb = rng.uniform(0.0, 1.0, (3, n))
    # The evaluated degree-0 colour is uniform in [0, 1]; the stored DC
    # coefficient is the value that evaluates to it (colour = c*Y00 + 0.5).
    y00 = 0.5 / math.sqrt(math.pi)
    sh = (rgb - 0.5) / y00
    g = Gaussians(mean.astype(np.float32), scale.astype(np.float32),
                  quat.astype(np.float32), opacity.astype(np.float32),
                  sh.astype(np.float32), 0)
    cam = Camera(np.eye(3).reshape(9), np.zeros(3), 150.0, 150.0, 64.0, 64.0,
                 128, 128, 0.2, (1.0, 1.0, 1.0)).as_f32()
    target = rng.uniform(0.0, 1.0, (3, 128, 128)).astype(np.float32)
    return g, cam, target


def config2(seed=2, n=1_000_000, width=1920, height=1080):
    """One partition cell: 1M Gaussians on a 200 m city patch, 1080p view."""
    g = city_gaussians(n, seed, size_m=200.0)
    cam = aerial_camera(width, height, 150.0)
    return g, cam


def config3(seed=3, n=200_000, size=800):
    """200k Gaussians on a 100 m patch, 800x800 camera at 75 m."""
    g = city_gaussians(n, seed, size_m=100.0)
    cam = aerial_camera(size, size, 75.0)
    return g, cam


CONFIG4_SIZES = (300_000, 500_000, 800_000, 1_000_000, 1_200_000, 1_600_000,
                 2_000_000, 2_500_000)


def config4(seed=4, sizes=CONFIG4_SIZES, width=1600, height=1066):
    """Eight cells of uneven Gaussian counts, one aerial view per cell."""
    cells = []
    for i, n in enumerate(sizes):
        g = city_gaussians(n, seed * 1000 + i, size_m=200.0)
        rng = np.random.default_rng(seed * 1000 + 100 + i)
        cam = aerial_camera(width, height, 150.0, yaw=float(rng.uniform(0, 2 * math.pi)))
        cells.append((g, cam))
    return cells


def merged_city(grid=10, cell_m=100.0, per_cell=200_000, seed=5, sh_degree=3):
    """A grid of city cells, each generated on its own, merged by keeping
    every cell's Gaussians that fall inside its un-expanded footprint and
    concatenating the cells.  Returns the merged set and per-cell AABBs
    [n_cells][6] = (xmin, ymin, zmin, xmax, ymax, zmax), each bounding the
    supports of its cell's Gaussians, plus cell offsets."""
    parts = []
    aabbs = []
    offsets = [0]
    half = grid * cell_m / 2.0
    for i in range(grid):
        for j in range(grid):
            cx = -half + (i + 0.5) * cell_m
            cz = -half + (j + 0.5) * cell_m
            g = city_gaussians(per_cell, seed * 100000 + i * grid + j,
                               size_m=cell_m, origin=(cx, cz), sh_degree=sh_degree)
            inside = ((g.mean[0] >= cx - cell_m / 2) & (g.mean[0] < cx + cell_m / 2) &
                      (g.mean[2] >= cz - cell_m / 2) & (g.mean[2] < cz + cell_m / 2))
            g = g.subset(np.nonzero(inside)[0])
            parts.append(g)
            # bound every Gaussian's alpha >= 1/255 support (at most
            # sqrt(2 ln 255) = 3.33 standard deviations from its mean)
            lo = g.mean.min(axis=1) - 3.5 * g.scale.max()
            hi = g.mean.max(axis=1) + 3.5 * g.scale.max()
            aabbs.append(np.concatenate([lo, hi]))
            offsets.append(offsets[-1] + g.n)
    merged = Gaussians(np.concatenate([p.mean for p in parts], axis=1),
                       np.concatenate([p.scale for p in parts], axis=1),
                       np.concatenate([p.quat for p in parts], axis=1),
                       np.concatenate([p.opacity for p in parts]),
                       np.concatenate([p.sh for p in parts], axis=1), sh_degree)
    return merged, np.asarray(aabbs, np.float32), np.asarray(offsets, np.int64)


SERVE_RESOLUTIONS = ((640, 480), (1280, 720), (1920, 1080), (3840, 2160))


def serve_trace(n_requests, rate_hz, seed=5, extent_m=1000.0,
                resolutions=SERVE_RESOLUTIONS, altitude=(80.0, 200.0),
                pitch_deg=(-90.0, -30.0)):
    """Poisson arrival trace of render requests over a square scene.

    Returns a list of (arrival_time_s, Camera)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for k in range(n_requests):
        w, h = resolutions[rng.integers(len(resolutions))]
        x, z = rng.uniform(-extent_m / 2, extent_m / 2, 2)
        y = rng.uniform(*altitude)
        yaw = rng.uniform(0, 2 * math.pi)
        pitch = math.radians(rng.uniform(*pitch_deg))
        pitch = max(pitch, math.radians(-89.5))
        out.append((float(t[k]), camera_from_pose((x, y, z), yaw, pitch, w, h)))
    return out


def small_city(n=20_000, seed=11, width=200, height=150, sh_degree=3,
               size_m=60.0, altitude=45.0, bg=(0.0, 0.0, 0.0), log_scale=(-1.6, 0.5)):
    """A reduced city scene for parity tests: ragged tile counts, SH
    degree 3, sizes the oracle finishes in seconds."""
    g = city_gaussians(n, seed, size_m=size_m, sh_degree=sh_degree,
                       log_scale=log_scale)
    cam = aerial_camera(width, height, altitude, bg=bg)
    return g, cam


def grad_image(cam: Camera, seed, kind="uniform"):
    """Seeded dLoss/dImage [3][H][W]: U[-1,1]/(3*Npix) or N(0,1)."""
    rng = np.random.default_rng(seed)
    shape = (3, cam.height, cam.width)
    if kind == "normal":
        return rng.standard_normal(shape).astype(np.float32)
    return (rng.uniform(-1.0, 1.0, shape) / (3.0 * cam.width * cam.height)).astype(np.float32)


def pixel_sample(width, height, stride=32, offset=None):
    """Stratified pixel sample: every `stride`-th row and column."""
    o = stride // 2 if offset is None else offset
    xs = np.arange(o, width, stride)
    ys = np.arange(o, height, stride)
    py, px = np.meshgrid(ys, xs, indexing="ij")
    return px.ravel().astype(np.int32), py.ravel().astype(np.int32)


# ---------------------------------------------------------- partitioning ---

def aerial_survey(n_views, seed, extent_m=1000.0, width=1152, height=864, altitude=(120.0, 180.0)):
    """A drone survey over a square site centred at the origin: camera
    positions on a jittered lawnmower grid at `altitude`, each view pitched
    -30..-90 deg with a random heading (the oblique captures of aerial
    datasets)."""
    rng = np.random.default_rng(seed)
    side = max(1, int(math.ceil(math.sqrt(n_views))))
    cams = []
    for k in range(n_views):
        i, j = divmod(k, side)
        if i % 2:
            j = side - 1 - j
        x = (i + 0.5) / side * extent_m - extent_m / 2 + rng.normal(0.0, 0.1 * extent_m / side)
        z = (j + 0.5) / side * extent_m - extent_m / 2 + rng.normal(0.0, 0.1 * extent_m / side)
        alt = rng.uniform(*altitude)
        pitch = math.radians(rng.uniform(-90.0, -30.0))
        yaw = rng.uniform(0.0, 2.0 * math.pi)
        if pitch < math.radians(-89.0):
            pitch = math.radians(-89.0)
        cams.append(camera_from_pose((x, alt, z), yaw, pitch, width, height))
    return cams


def sfm_points(n, seed, extent_m=1000.0):
    """A sparse point cloud of the city over the same site: [n][3] float32
    world positions on the ground and the building tops."""
    g = city_gaussians(n, seed, size_m=extent_m, sh_degree=0)
    return np.ascontiguousarray(g.mean.T, np.float32)
