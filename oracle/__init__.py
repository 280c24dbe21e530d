"""FP64 CPU oracle for the Gaussian tile rasterizer -- TEST INFRASTRUCTURE.

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's `cpu_baseline`
leg may import this package.  The product path never does: it shares no code
with the oracle, and must fail loudly when its HIP library is missing.

The arithmetic lives in `gs_oracle.c` (plain C, FP64, OpenMP over pixels);
this module only marshals NumPy arrays through ctypes.  What the oracle
computes follows VastGaussian (arXiv 2402.17427) section 3: 3D Gaussians
(position, anisotropic covariance, opacity, SH colour) are projected to 2D
Gaussians by EWA splatting and alpha-blended front to back; the renderer is
differentiable and the Gaussians are optimised by gradients.  The
image-formation constants the paper leaves to 3DGS (section 5.1) are the
readings listed at the top of `gs_oracle.c`.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# relative windows around the discontinuous decisions (alpha vs 1/255 and
# 0.99, T vs 1e-4, power vs 0) inside which a pixel is flagged ambiguous
DEFAULT_EPS = (1e-4, 1e-3, 1e-5)


_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")


def build_sanitized() -> str:
    """The oracle built with clang under AddressSanitizer and
    UndefinedBehaviorSanitizer (no OpenMP: one sanitizer runtime, clang's,
    serves it and the sanitized rasterizer library in one process); loaded
    instead of the regular build when GS_ORACLE_LIB names it."""
    clang = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib", "llvm", "bin", "clang")
    tmp = _LIB_SAN + ".tmp"
    subprocess.check_call([clang, "-O1", "-g", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-Wall",
                           "-Wno-unknown-pragmas", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_SAN)
    return _LIB_SAN


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def build_planted(macro: str, out_dir: str) -> str:
    """Compile a copy of the oracle with one planted mistake switched on
    (`-D<macro>`) into `out_dir`; tests load it with `planted_library` to show
    that their pins catch the mistake."""
    path = os.path.join(out_dir, f"liboracle_{macro.lower()}.so")
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                           f"-D{macro}", "-o", path, _SRC, "-lm"])
    return path


@contextlib.contextmanager
def planted_library(path):
    """Route the oracle calls made inside the block through the library at
    `path` (a planted build), then back to the regular one."""
    global _lib
    prev = _lib
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = prev


def lib():
    global _lib
    if _lib is None:
        alt = os.environ.get("GS_ORACLE_LIB")
        if alt:
            _lib = _load(alt)
        else:
            if not os.path.exists(_LIB):
                build()
            _lib = _load(_LIB)
    return _lib


def _load(path):
    L = C.CDLL(path)
    P = C.c_void_p
    i64 = C.c_int64
    L.orc_project.argtypes = [i64, i64, C.c_int] + [P] * 6 + [P] * 8
    L.orc_project.restype = C.c_int
    L.orc_render.argtypes = [i64, i64, C.c_int] + [P] * 6 + [i64, P, P, P] + [P] * 5
    L.orc_render.restype = C.c_int
    L.orc_backward.argtypes = [i64, i64, C.c_int] + [P] * 6 + [P, i64, P, P, P] + [P] * 8
    L.orc_backward.restype = C.c_int
    L.orc_bin.argtypes = [i64, i64, C.c_int] + [P] * 6 + [C.c_int, C.c_int, C.c_double, P, P, i64,
                                                           P, P, P, P, P]
    L.orc_bin.restype = C.c_int64
    L.orc_render_tiled.argtypes = [i64, i64, C.c_int] + [P] * 6 + [C.c_int, C.c_int, P, P, P, P]
    L.orc_render_tiled.restype = C.c_int
    L.orc_sh_basis.argtypes = [P, P]
    L.orc_sh_basis_grad.argtypes = [P, P]
    L.orc_num_threads.restype = C.c_int
    L.orc_set_num_threads.argtypes = [C.c_int]
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def camera_vec(cam) -> np.ndarray:
    """22 doubles: R[9], t[3], fx, fy, cx, cy, W, H, near, bg[3]."""
    v = np.zeros(22, np.float64)
    v[0:9] = np.asarray(cam.R, np.float64).reshape(9)
    v[9:12] = np.asarray(cam.t, np.float64).reshape(3)
    v[12:16] = [cam.fx, cam.fy, cam.cx, cam.cy]
    v[16:18] = [cam.width, cam.height]
    v[18] = cam.near
    v[19:22] = cam.bg
    return v


class _G:
    """Gaussian set widened to float64 (the oracle's input form)."""

    def __init__(self, g):
        self.n = g.mean.shape[1]
        self.deg = g.sh_degree
        self.mean, self.scale, self.quat = _d(g.mean), _d(g.scale), _d(g.quat)
        self.opacity, self.sh = _d(g.opacity), _d(g.sh)

    def args(self):
        return (self.n, self.n, self.deg, _p(self.mean), _p(self.scale), _p(self.quat),
                _p(self.opacity), _p(self.sh))


def project(g, cam):
    """Per-Gaussian FP64 projection: dict of valid, uv, conic, cov, rgb,
    depth, ext, pxrect."""
    G = _G(g)
    n = G.n
    out = dict(valid=np.zeros(n, np.int32), uv=np.zeros((n, 2)), conic=np.zeros((n, 3)),
               cov=np.zeros((n, 3)), rgb=np.zeros((n, 3)), depth=np.zeros(n),
               ext=np.zeros((n, 2)), pxrect=np.zeros((n, 4), np.int32))
    cv = camera_vec(cam)
    rc = lib().orc_project(*G.args(), _p(cv), *[_p(out[k]) for k in
                           ("valid", "uv", "conic", "cov", "rgb", "depth", "ext", "pxrect")])
    if rc:
        raise ValueError(f"orc_project failed ({rc})")
    return out


def render(g, cam, px=None, py=None, eps=DEFAULT_EPS):
    """All-pairs FP64 render.  Full frame (image [3][H][W]) when px is None,
    else values at the listed pixels ([npix][3]).  Returns dict image,
    final_T, last_id, nblend, flags."""
    G = _G(g)
    cv = camera_vec(cam)
    if px is None:
        npix = cam.width * cam.height
        pxa = pya = None
    else:
        pxa = np.ascontiguousarray(px, np.int32)
        pya = np.ascontiguousarray(py, np.int32)
        npix = pxa.size
    img = np.zeros((npix, 3))
    fT = np.zeros(npix)
    last = np.zeros(npix, np.int64)
    nb = np.zeros(npix, np.int64)
    fl = np.zeros(npix, np.int32)
    e = np.asarray(eps, np.float64)
    rc = lib().orc_render(*G.args(), _p(cv), npix, _p(pxa), _p(pya), _p(e), _p(img), _p(fT),
                          _p(last), _p(nb), _p(fl))
    if rc:
        raise ValueError(f"orc_render failed ({rc})")
    if px is None:
        H, W = cam.height, cam.width
        return dict(image=img.reshape(H, W, 3).transpose(2, 0, 1).copy(), final_T=fT.reshape(H, W),
                    last_id=last.reshape(H, W), nblend=nb.reshape(H, W), flags=fl.reshape(H, W))
    return dict(image=img, final_T=fT, last_id=last, nblend=nb, flags=fl)


def backward(g, cam, dimg, px=None, py=None, eps=DEFAULT_EPS):
    """Analytic FP64 gradient of L = sum(dimg * image).  dimg: [3][H][W].
    Returns dict mean, scale, quat, opacity, sh (input layout), g2d [n][9],
    flags (per pixel), touch [n]."""
    G = _G(g)
    n, K = G.n, (G.deg + 1) ** 2
    cv = camera_vec(cam)
    dimg = _d(dimg)
    assert dimg.shape == (3, cam.height, cam.width)
    if px is None:
        npix = cam.width * cam.height
        pxa = pya = None
    else:
        pxa = np.ascontiguousarray(px, np.int32)
        pya = np.ascontiguousarray(py, np.int32)
        npix = pxa.size
    out = dict(mean=np.zeros((3, n)), scale=np.zeros((3, n)), quat=np.zeros((4, n)),
               opacity=np.zeros(n), sh=np.zeros((3 * K, n)), g2d=np.zeros((n, 9)),
               flags=np.zeros(npix, np.int32), touch=np.zeros(n, np.int32))
    e = np.asarray(eps, np.float64)
    rc = lib().orc_backward(*G.args(), _p(cv), _p(dimg), npix, _p(pxa), _p(pya), _p(e),
                            *[_p(out[k]) for k in ("mean", "scale", "quat", "opacity", "sh", "g2d",
                                                   "flags", "touch")])
    if rc:
        raise ValueError(f"orc_backward failed ({rc})")
    return out


def bin(g, cam, tile_w=16, tile_h=16, eps_px=1e-6):
    """Tile binning from the FP64 projection: dict keys (u64), vals (u32),
    ranges [T][2], tiles_touched, trect [n][4], zbits, amb."""
    G = _G(g)
    n = G.n
    cv = camera_vec(cam)
    tt = np.zeros(n, np.uint32)
    tr = np.zeros((n, 4), np.int32)
    zb = np.zeros(n, np.uint32)
    amb = np.zeros(n, np.int32)
    total = lib().orc_bin(*G.args(), _p(cv), tile_w, tile_h, eps_px, None, None, 0, None,
                          _p(tt), _p(tr), _p(zb), _p(amb))
    if total < 0:
        raise ValueError(f"orc_bin failed ({total})")
    ntx = (cam.width + tile_w - 1) // tile_w
    nty = (cam.height + tile_h - 1) // tile_h
    keys = np.zeros(max(total, 1), np.uint64)
    vals = np.zeros(max(total, 1), np.uint32)
    ranges = np.zeros((ntx * nty, 2), np.uint32)
    t2 = lib().orc_bin(*G.args(), _p(cv), tile_w, tile_h, eps_px, _p(keys), _p(vals), total,
                       _p(ranges), None, None, None, None)
    if t2 != total:
        raise ValueError("orc_bin pair count changed")
    return dict(keys=keys[:total], vals=vals[:total], ranges=ranges, tiles_touched=tt, trect=tr,
                zbits=zb, amb=amb, n_tiles=(ntx, nty))


def render_tiled(g, cam, vals, ranges, tile_w=16, tile_h=16):
    """Re-evaluate the image walking only each pixel's tile list."""
    G = _G(g)
    cv = camera_vec(cam)
    vals = np.ascontiguousarray(vals, np.uint32)
    ranges = np.ascontiguousarray(ranges, np.uint32)
    npix = cam.width * cam.height
    img = np.zeros((npix, 3))
    fT = np.zeros(npix)
    rc = lib().orc_render_tiled(*G.args(), _p(cv), tile_w, tile_h, _p(vals), _p(ranges), _p(img), _p(fT))
    if rc:
        raise ValueError("orc_render_tiled failed")
    H, W = cam.height, cam.width
    return img.reshape(H, W, 3).transpose(2, 0, 1).copy(), fT.reshape(H, W)


def sh_basis(d):
    d = _d(d).reshape(3)
    Y = np.zeros(16)
    lib().orc_sh_basis(_p(d), _p(Y))
    return Y


def sh_basis_grad(d):
    d = _d(d).reshape(3)
    dY = np.zeros((16, 3))
    lib().orc_sh_basis_grad(_p(d), _p(dY))
    return dY


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's later OpenMP regions."""
    lib().orc_set_num_threads(int(n))
