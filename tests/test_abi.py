"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every function include/gs.h declares, and rejects bad arguments on the host
before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_2402_17427_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^[A-Za-z_][\w \*]*?\b(gs_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("gs_project", "gs_bin_sort", "gs_render_fwd", "gs_render_bwd"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = N.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_abi_version_and_error_strings():
    lib = N.lib()
    assert lib.gs_abi_version() == 2
    nbytes = C.c_size_t(0)
    assert lib.gs_bin_sort_workspace(-1, 10, 4, C.byref(nbytes)) == N.GS_ERR_INVALID
    assert b"bad sizes" in lib.gs_last_error()
    # up to 32768 tiles (direct placement): the 8-byte placed pairs of the
    # capacity and at least one count-matrix row of the tiles
    assert lib.gs_bin_sort_workspace(1000, 4000, 64, C.byref(nbytes)) == N.GS_OK
    assert nbytes.value >= 4000 * 8 + 64 * 4
    # above (emission + radix sort): the emitted 8-byte keys and 4-byte
    # values of the capacity
    assert lib.gs_bin_sort_workspace(1000, 4000, 40000, C.byref(nbytes)) == N.GS_OK
    assert nbytes.value >= 4000 * 12


def test_host_validation_rejects_bad_descriptors_without_a_device():
    lib = N.lib()
    cam = N.gs_camera()
    cam.width, cam.height, cam.fx, cam.fy = 64, 64, 100.0, 100.0
    g = N.gs_gaussians()
    g.n, g.ld, g.sh_degree = 10, 5, 0          # ld < n
    proj = N.gs_proj()
    assert lib.gs_project(C.byref(g), C.byref(cam), None, C.byref(proj), None) == N.GS_ERR_INVALID
    g.ld = 10
    g.sh_degree = 7
    assert lib.gs_project(C.byref(g), C.byref(cam), None, C.byref(proj), None) == N.GS_ERR_INVALID
    g.sh_degree = 0
    cam.width = 0
    assert lib.gs_project(C.byref(g), C.byref(cam), None, C.byref(proj), None) == N.GS_ERR_INVALID
    cam.width = 64
    # NULL planes
    assert lib.gs_project(C.byref(g), C.byref(cam), None, C.byref(proj), None) == N.GS_ERR_INVALID
    opts = N.make_opts(24, 16)
    g.n = 0
    assert lib.gs_project(C.byref(g), C.byref(cam), C.byref(opts), C.byref(proj), None) == N.GS_ERR_UNSUPPORTED
    bins = N.gs_bins()
    bins.pair_capacity = 1 << 31
    assert lib.gs_render_fwd(C.byref(proj), C.byref(bins), C.byref(cam), None, None, None, None,
                             None) == N.GS_ERR_INVALID


def test_backward_workspace_query_and_validation_without_a_device():
    """gs_render_bwd_workspace sizes the per-pair gradient slots (36 bytes
    per pair of capacity); gs_render_bwd rejects a missing, short or
    misaligned workspace and a NULL bins.first before any launch (the
    device pointers below are never dereferenced)."""
    lib = N.lib()
    fake = 1 << 20   # 256-byte aligned stand-in for device buffers
    bins = N.gs_bins()
    bins.keys, bins.vals, bins.first = fake, fake, fake
    bins.ranges, bins.pair_count, bins.status = fake, fake, fake
    bins.pair_capacity = 1000
    nbytes = C.c_size_t(0)
    assert lib.gs_render_bwd_workspace(C.byref(bins), C.byref(nbytes)) == N.GS_OK
    # 36 B of gradient slots per pair, then a tile order of at most one entry per pair and its count
    assert 40 * 1000 <= nbytes.value <= 40 * 1000 + 516
    assert lib.gs_render_bwd_workspace(None, C.byref(nbytes)) == N.GS_ERR_INVALID

    g = N.gs_gaussians()
    g.n, g.ld, g.sh_degree = 10, 10, 0
    g.mean = g.scale = g.quat = g.opacity = g.sh = fake
    cam = N.gs_camera()
    cam.width, cam.height, cam.fx, cam.fy, cam.near_z = 64, 64, 100.0, 100.0, 0.2
    cam.R[0] = cam.R[4] = cam.R[8] = 1.0
    proj = N.gs_proj()
    proj.rec, proj.depth, proj.rect, proj.tiles_touched = fake, fake, fake, fake
    out = N.gs_grads()
    out.ld = 10
    out.mean = out.scale = out.quat = out.opacity = out.sh = out.grad2d = fake

    def bwd(ws, ws_bytes):
        return lib.gs_render_bwd(C.byref(g), C.byref(cam), None, C.byref(proj), C.byref(bins), fake, fake, fake,
                                 C.byref(out), ws, ws_bytes, None)

    assert bwd(None, 0) == N.GS_ERR_INVALID
    assert b"workspace" in lib.gs_last_error()
    assert bwd(fake, nbytes.value - 4) == N.GS_ERR_INVALID
    assert bwd(fake + 4, nbytes.value) == N.GS_ERR_INVALID
    assert b"aligned" in lib.gs_last_error()
    bins.first = None
    assert bwd(fake, 36 * 1000) == N.GS_ERR_INVALID
    assert b"first" in lib.gs_last_error()


def test_loss_workspace_query_and_validation_without_a_device():
    """gs_loss_workspace sizes one (float, float) partial per 32 x 32 tile
    of every channel; gs_loss rejects bad shapes, NULL buffers, a missing
    d_image_l1 for the Eq. 3 form, a non-finite lambda and a short or
    misaligned workspace before any launch."""
    lib = N.lib()
    nbytes = C.c_size_t(0)
    assert lib.gs_loss_workspace(3, 1920, 1080, C.byref(nbytes)) == N.GS_OK
    assert nbytes.value == 8 * 3 * 60 * 34
    assert lib.gs_loss_workspace(3, 33, 1, C.byref(nbytes)) == N.GS_OK
    assert nbytes.value == 8 * 3 * 2
    for bad in ((0, 8, 8), (3, 0, 8), (3, 8, -1)):
        assert lib.gs_loss_workspace(*bad, C.byref(nbytes)) == N.GS_ERR_INVALID
    assert lib.gs_loss_workspace(3, 8, 8, None) == N.GS_ERR_INVALID
    fake = 1 << 20
    need = 8 * 3

    def loss(img=fake, img_l1=None, tgt=fake, c=3, w=8, h=8, lam=0.2, out=fake, d=fake, d1=None, ws=fake,
             ws_bytes=need):
        return lib.gs_loss(img, img_l1, tgt, c, w, h, C.c_float(lam), out, d, d1, ws, ws_bytes, None)

    assert loss(img=None) == N.GS_ERR_INVALID
    assert loss(tgt=None) == N.GS_ERR_INVALID
    assert loss(out=None) == N.GS_ERR_INVALID
    assert loss(d=None) == N.GS_ERR_INVALID
    assert loss(c=0) == N.GS_ERR_INVALID
    assert loss(img_l1=fake) == N.GS_ERR_INVALID
    assert b"d_image_l1" in lib.gs_last_error()
    assert loss(lam=float("nan")) == N.GS_ERR_INVALID
    assert loss(ws_bytes=need - 1) == N.GS_ERR_INVALID
    assert b"workspace" in lib.gs_last_error()
    assert loss(ws=fake + 4) == N.GS_ERR_INVALID
    assert b"aligned" in lib.gs_last_error()


def test_loss_noalloc_validation_without_a_device():
    """gs_loss_noalloc checks its arguments like gs_loss and rejects an
    image whose partial sums exceed its fixed scratch (GS_ERR_CAPACITY)
    before any device call."""
    lib = N.lib()
    fake = 1 << 20

    def call(img=fake, img_l1=None, tgt=fake, c=3, w=8, h=8, lam=0.2, out=fake, d=fake, d1=None):
        return lib.gs_loss_noalloc(img, img_l1, tgt, c, w, h, C.c_float(lam), out, d, d1, None)

    assert call(img=None) == N.GS_ERR_INVALID
    assert call(d=None) == N.GS_ERR_INVALID
    assert call(c=0) == N.GS_ERR_INVALID
    assert call(img_l1=fake) == N.GS_ERR_INVALID
    assert call(lam=float("inf")) == N.GS_ERR_INVALID
    # 3 x 256 x 256 tiles of 32 x 32: more partials than the scratch holds
    assert call(w=8192, h=8192) == N.GS_ERR_CAPACITY
    assert b"partial sums" in lib.gs_last_error()


def test_adam_step_validation_without_a_device():
    """gs_adam_step rejects NULL descriptors and buffers, ld < n, a bad SH
    degree and out-of-range hyper-parameters before any launch (the device
    pointers below are never dereferenced)."""
    lib = N.lib()
    fake = 1 << 20
    p = N.gs_params()
    p.n, p.ld, p.sh_degree = 10, 10, 3
    p.mean = p.log_scale = p.quat = p.logit_opacity = p.sh = fake
    st = N.gs_adam_state()
    st.m = st.v = st.grad_accum = st.visible_count = fake
    gr = N.gs_grads()
    gr.ld = 10
    gr.mean = gr.scale = gr.quat = gr.opacity = gr.sh = gr.grad2d = fake

    def cfg(**kw):
        c = N.gs_adam_config()
        c.lr_mean = c.lr_scale = c.lr_quat = c.lr_opacity = c.lr_sh_dc = c.lr_sh_rest = 1e-3
        c.beta1, c.beta2, c.eps, c.step = 0.9, 0.999, 1e-15, 1
        for k, v in kw.items():
            setattr(c, k, v)
        return c

    def step(c, pp=p, s=st, g=gr, so=fake, oo=fake, tiles=fake):
        return lib.gs_adam_step(C.byref(pp) if pp is not None else None, so, oo,
                                C.byref(s) if s is not None else None, C.byref(g) if g is not None else None,
                                tiles, None, C.byref(c) if c is not None else None, None)

    assert step(None) == N.GS_ERR_INVALID
    assert step(cfg(), pp=None) == N.GS_ERR_INVALID
    assert step(cfg(), s=None) == N.GS_ERR_INVALID
    assert step(cfg(), g=None) == N.GS_ERR_INVALID
    assert step(cfg(), so=None) == N.GS_ERR_INVALID
    for bad in (dict(beta1=1.0), dict(beta2=-0.1), dict(eps=-1.0), dict(step=0), dict(lr_quat=float("inf"))):
        assert step(cfg(**bad)) == N.GS_ERR_INVALID, bad
    p.ld = 5
    assert step(cfg()) == N.GS_ERR_INVALID
    p.ld, p.sh_degree = 10, 4
    assert step(cfg()) == N.GS_ERR_INVALID
    p.sh_degree = 3
    gr.ld = 9
    assert step(cfg()) == N.GS_ERR_INVALID
    gr.ld = 10
    st.grad_accum = None
    assert step(cfg()) == N.GS_ERR_INVALID
    assert b"statistics" in lib.gs_last_error()
