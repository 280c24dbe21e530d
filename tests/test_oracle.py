"""Pins of the FP64 oracle against facts fixed outside it.

Each test checks the oracle against something other than its own formulas:
closed forms of special cases, a library routine (SciPy rotations and
spherical harmonics, a finite-difference Jacobian), brute force on tiny
inputs, the compositing invariants, and central finite differences of its
own forward for the analytic gradient.  What is pinned follows VastGaussian
(arXiv 2402.17427) section 3: EWA projection of 3D Gaussians, SH colour,
tile assignment, depth sort and front-to-back alpha blending, differentiable
w.r.t. every Gaussian parameter.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy import special

import oracle
from gen import scenes

Y00 = 0.5 / math.sqrt(math.pi)


def one_gaussian(mu, s, q, o, rgb, deg=0):
    K = (deg + 1) ** 2
    sh = np.zeros((3 * K, 1))
    for c in range(3):
        sh[c * K, 0] = (rgb[c] - 0.5) / Y00
    return scenes.Gaussians(np.asarray(mu, np.float64).reshape(3, 1), np.asarray(s, np.float64).reshape(3, 1),
                            np.asarray(q, np.float64).reshape(4, 1), np.asarray([o], np.float64), sh, deg)


def stack(*gs):
    return scenes.Gaussians(np.concatenate([g.mean for g in gs], 1), np.concatenate([g.scale for g in gs], 1),
                            np.concatenate([g.quat for g in gs], 1), np.concatenate([g.opacity for g in gs]),
                            np.concatenate([g.sh for g in gs], 1), gs[0].sh_degree)


def ident_cam(W=64, H=48, f=100.0, bg=(0.2, 0.3, 0.4)):
    return scenes.Camera(np.eye(3).reshape(9), np.zeros(3), f, f, W / 2, H / 2, W, H, 0.2, bg)


def pixel_grid(cam):
    ys, xs = np.meshgrid(np.arange(cam.height) + 0.5, np.arange(cam.width) + 0.5, indexing="ij")
    return xs, ys


def closed_alpha(o, quad):
    a = np.minimum(0.99, o * np.exp(-0.5 * quad))
    return np.where(a >= 1 / 255, a, 0.0)


# ------------------------------------------------------------- projection --

def test_single_isotropic_gaussian_closed_form():
    """Isotropic Gaussian on the optical axis: the 2D covariance is
    ((f sigma / z)^2 + 0.3) I and each pixel is rgb a + (1 - a) bg."""
    cam = ident_cam()
    sig, z, o, rgb = 0.05, 4.0, 0.8, (0.9, 0.1, 0.5)
    g = one_gaussian((0, 0, z), (sig, sig, sig), (1, 0, 0, 0), o, rgb)
    var = (cam.fx * sig / z) ** 2 + 0.3
    r = oracle.render(g, cam)
    xs, ys = pixel_grid(cam)
    rho2 = (xs - cam.cx) ** 2 + (ys - cam.cy) ** 2
    a = closed_alpha(o, rho2 / var)
    for c in range(3):
        want = rgb[c] * a + (1 - a) * cam.bg[c]
        np.testing.assert_allclose(r["image"][c], want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["final_T"], 1 - a, atol=1e-12)
    p = oracle.project(g, cam)
    np.testing.assert_allclose(p["cov"][0], [var, 0, var], rtol=1e-12, atol=1e-12)


def test_rotated_camera_isotropic_closed_form():
    """Same closed form through a general look-at camera (world rotation)."""
    cam = scenes.look_at((3.0, 5.0, -2.0), (1.0, 0.5, 4.0), 80, 60, hfov_deg=50, bg=(0, 0, 0))
    eye = np.array([3.0, 5.0, -2.0])
    Rm = np.asarray(cam.R, np.float64).reshape(3, 3)
    eye = -Rm.T @ np.asarray(cam.t, np.float64)       # camera centre of the float32 camera
    d = Rm[2]                                          # optical axis in world
    z = 6.0
    mu = eye + z * d
    sig, o = 0.08, 0.6
    g = one_gaussian(mu, (sig,) * 3, (0.3, -0.2, 0.5, 0.1), o, (0.7, 0.2, 0.4))
    p = oracle.project(g, cam)
    var = (cam.fx * sig / z) ** 2 + 0.3
    # the camera rotation is stored in float32, orthonormal only to ~1e-7
    np.testing.assert_allclose(p["cov"][0], [var, 0, var], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(p["uv"][0], [cam.cx, cam.cy], atol=1e-5)
    np.testing.assert_allclose(p["depth"][0], z, rtol=1e-7)


def test_anisotropic_rotated_about_axis_closed_form():
    """Rotation by theta about the optical axis: covariance
    (f/z)^2 R2 diag(sx^2, sy^2) R2^T + 0.3 I."""
    cam = ident_cam(f=120.0)
    th, z = 0.7, 5.0
    sx, sy, sz = 0.09, 0.03, 0.2
    q = (math.cos(th / 2), 0, 0, math.sin(th / 2))
    g = one_gaussian((0, 0, z), (sx, sy, sz), q, 0.9, (0.3, 0.6, 0.9))
    R2 = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    S2 = (cam.fx / z) ** 2 * R2 @ np.diag([sx * sx, sy * sy]) @ R2.T + 0.3 * np.eye(2)
    p = oracle.project(g, cam)
    np.testing.assert_allclose(p["cov"][0], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-12, atol=1e-12)
    Q = np.linalg.inv(S2)
    np.testing.assert_allclose(p["conic"][0], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-10)
    r = oracle.render(g, cam)
    xs, ys = pixel_grid(cam)
    dx, dy = xs - cam.cx, ys - cam.cy
    quad = Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy
    a = closed_alpha(0.9, quad)
    np.testing.assert_allclose(r["image"][1], 0.6 * a + (1 - a) * cam.bg[1], atol=1e-12)


def _numeric_jacobian(cam, t, h=1e-6):
    def proj(tt):
        return np.array([cam.fx * tt[0] / tt[2] + cam.cx, cam.fy * tt[1] / tt[2] + cam.cy])
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h * max(1.0, abs(t[k]))
        J[:, k] = (proj(t + e) - proj(t - e)) / (2 * e[k])
    return J


def test_ewa_covariance_matches_library_rotation_and_numeric_jacobian():
    """Off-axis Gaussians: 2D covariance = J W Sigma W^T J^T + 0.3 I with
    Sigma from SciPy's rotation of the quaternion and J the numerical
    Jacobian of the pinhole map at the (unclamped) centre."""
    rng = np.random.default_rng(7)
    cam = scenes.look_at((0, 10, -10), (0, 0, 0), 160, 120, hfov_deg=60)
    n = 50
    Rm = np.asarray(cam.R, np.float64).reshape(3, 3)
    tv = np.asarray(cam.t, np.float64)
    mean = rng.uniform(-3, 3, (3, n))
    g = scenes.Gaussians(mean, np.exp(rng.normal(-2, 0.5, (3, n))), rng.normal(size=(4, n)),
                         rng.uniform(0.2, 0.9, n), rng.normal(size=(3, n)), 0)
    p = oracle.project(g, cam)
    checked = 0
    for i in range(n):
        t = Rm @ mean[:, i] + tv
        limx = 1.3 * (cam.width / 2) / cam.fx
        limy = 1.3 * (cam.height / 2) / cam.fy
        if t[2] <= 0.2 or abs(t[0] / t[2]) > limx or abs(t[1] / t[2]) > limy:
            continue
        q = g.quat[:, i]
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()   # SciPy is scalar-last
        Sig = Rq @ np.diag(g.scale[:, i] ** 2) @ Rq.T
        J = _numeric_jacobian(cam, t)
        S2 = J @ Rm @ Sig @ Rm.T @ J.T + 0.3 * np.eye(2)
        np.testing.assert_allclose(p["cov"][i], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-6, atol=1e-9)
        u = cam.fx * t[0] / t[2] + cam.cx
        np.testing.assert_allclose(p["uv"][i, 0], u, rtol=1e-12)
        np.testing.assert_allclose(p["depth"][i], t[2], rtol=1e-12)
        checked += 1
    assert checked > 20


def test_fov_clamp_freezes_covariance_beyond_limit():
    """Beyond 1.3x the half field of view the Jacobian is taken at the
    clamped ray, so moving further out along x at fixed depth leaves the 2D
    covariance unchanged while the centre keeps moving."""
    cam = ident_cam(W=64, H=64, f=64.0)
    z = 4.0
    lim = 1.3 * 32 / 64.0
    xs = [lim * z * 1.1, lim * z * 1.5, lim * z * 3.0]
    gs = [one_gaussian((x, 0.2, z), (0.5, 0.3, 0.2), (0.9, 0.1, 0.3, 0.2), 0.9, (0.5, 0.5, 0.5)) for x in xs]
    p = oracle.project(stack(*gs), cam)
    np.testing.assert_allclose(p["cov"][0], p["cov"][1], rtol=1e-12)
    np.testing.assert_allclose(p["cov"][0], p["cov"][2], rtol=1e-12)
    assert p["uv"][2, 0] > p["uv"][1, 0] > p["uv"][0, 0]


def test_culling_rules():
    """Near plane, opacity below 1/255 and off-image Gaussians are culled;
    non-finite inputs are culled."""
    cam = ident_cam()
    gs = [one_gaussian((0, 0, 0.1), (0.05,) * 3, (1, 0, 0, 0), 0.9, (1, 1, 1)),      # behind near
          one_gaussian((0, 0, 3.0), (0.05,) * 3, (1, 0, 0, 0), 0.5 / 255, (1, 1, 1)),  # too transparent
          one_gaussian((50, 0, 3.0), (0.05,) * 3, (1, 0, 0, 0), 0.9, (1, 1, 1)),     # off image
          one_gaussian((0, 0, 3.0), (np.nan, 0.05, 0.05), (1, 0, 0, 0), 0.9, (1, 1, 1)),
          one_gaussian((0, 0, 3.0), (0.05,) * 3, (0, 0, 0, 0), 0.9, (1, 1, 1)),       # zero quaternion
          one_gaussian((0, 0, 3.0), (0.05,) * 3, (1, 0, 0, 0), 0.9, (1, 0, 0))]
    p = oracle.project(stack(*gs), cam)
    assert list(p["valid"]) == [0, 0, 0, 0, 0, 1]


# -------------------------------------------------------------- colour --

def _quadrature(nt=12, nph=24):
    x, w = np.polynomial.legendre.leggauss(nt)
    ph = np.arange(nph) * 2 * np.pi / nph
    ct, PH = np.meshgrid(x, ph, indexing="ij")
    W = np.repeat(w[:, None], nph, 1) * (2 * np.pi / nph)
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(PH), st * np.sin(PH), ct], -1).reshape(-1, 3)
    return d, W.ravel(), np.arccos(ct).ravel(), PH.ravel()


def test_sh_basis_orthonormal_by_quadrature():
    """The 16 real SH basis functions are orthonormal on the sphere, which
    pins every normalisation constant (not the signs)."""
    d, w, _, _ = _quadrature()
    Y = np.stack([oracle.sh_basis(v) for v in d])
    Gm = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(Gm, np.eye(16), atol=1e-12)


def test_sh_basis_matches_scipy_up_to_sign():
    """Each basis function equals +-1 times SciPy's real spherical harmonic
    of the same (l, m), with a sign that is constant over the sphere; the
    sign pattern itself is a convention (parity unpinned)."""
    d, _, theta, phi = _quadrature(6, 9)
    Y = np.stack([oracle.sh_basis(v) for v in d])
    for l in range(4):
        for m in range(-l, l + 1):
            j = l * l + l + m
            Yc = special.sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                ref = math.sqrt(2) * (-1) ** m * Yc.real
            elif m < 0:
                ref = math.sqrt(2) * (-1) ** m * Yc.imag
            else:
                ref = Yc.real
            s = np.sign(np.dot(ref, Y[:, j]))
            np.testing.assert_allclose(Y[:, j], s * ref, atol=1e-12)


def test_sh_basis_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    for _ in range(5):
        d = rng.normal(size=3)
        dY = oracle.sh_basis_grad(d)
        for k in range(3):
            e = np.zeros(3)
            e[k] = 1e-6
            fd = (oracle.sh_basis(d + e) - oracle.sh_basis(d - e)) / 2e-6
            np.testing.assert_allclose(dY[:, k], fd, rtol=1e-6, atol=1e-8)


def test_dc_colour_closed_form_and_clamp():
    """Degree 0: rgb = k0 / (2 sqrt(pi)) + 0.5, clamped below at 0 only."""
    cam = ident_cam()
    g = one_gaussian((0, 0, 3), (0.05,) * 3, (1, 0, 0, 0), 0.9, (0.25, 1.7, 0.0))
    g.sh[2, 0] = -3.0          # raw colour -3 * Y00 + 0.5 < 0 -> clamped to 0
    p = oracle.project(g, cam)
    np.testing.assert_allclose(p["rgb"][0], [0.25, 1.7, 0.0], atol=1e-14)


# ------------------------------------------------------------ compositing --

def test_two_gaussian_stack_closed_form_and_depth_order():
    """Two Gaussians: c1 a1 + c2 a2 (1 - a1) + bg (1-a1)(1-a2), nearer first
    regardless of index order.  For an isotropic Gaussian at camera-space
    (x, y, z) the EWA covariance is s^2 (f/z)^2 [[1 + x'^2, x'y'], [x'y',
    1 + y'^2]] + 0.3 I with x' = x/z, y' = y/z (J J^T of the pinhole map)."""
    cam = ident_cam()
    near = one_gaussian((0, 0, 3.0), (0.06,) * 3, (1, 0, 0, 0), 0.7, (1.0, 0.0, 0.0))
    far = one_gaussian((0.1, 0.05, 5.0), (0.12,) * 3, (1, 0, 0, 0), 0.6, (0.0, 1.0, 0.0))
    xs, ys = pixel_grid(cam)

    def iso_alpha(t, s, o):
        xp, yp = t[0] / t[2], t[1] / t[2]
        S2 = (s * cam.fx / t[2]) ** 2 * np.array([[1 + xp * xp, xp * yp], [xp * yp, 1 + yp * yp]]) + 0.3 * np.eye(2)
        Q = np.linalg.inv(S2)
        dx, dy = xs - (cam.fx * xp + cam.cx), ys - (cam.fy * yp + cam.cy)
        return closed_alpha(o, Q[0, 0] * dx * dx + 2 * Q[0, 1] * dx * dy + Q[1, 1] * dy * dy)

    a1 = iso_alpha((0, 0, 3.0), 0.06, 0.7)
    a2 = iso_alpha((0.1, 0.05, 5.0), 0.12, 0.6)
    for order in ((near, far), (far, near)):
        r = oracle.render(stack(*order), cam)
        for c, (c1, c2) in enumerate(((1, 0), (0, 1), (0, 0))):
            want = c1 * a1 + c2 * a2 * (1 - a1) + cam.bg[c] * (1 - a1) * (1 - a2)
            np.testing.assert_allclose(r["image"][c], want, rtol=0, atol=1e-12)


def test_stop_rule_ends_the_walk_at_the_crossing_gaussian():
    """On-axis Gaussians with alphas a1, a2 (T2 = (1-a1)(1-a2) just above
    1e-4), a saturated third that would drop T below 1e-4 and a faint fourth
    that alone would not: the walk stops at the third, so neither the third
    nor the fourth is blended and the pixel is c1 a1 + c2 a2 (1-a1) + bg T2."""
    cam = ident_cam(W=16, H=16, f=50)
    specs = ((3, 0.999, (1, 0, 0)), (4, 0.985, (0, 1, 0)), (5, 0.999, (0, 0, 1)), (6, 0.3, (1, 1, 1)))
    gs = [one_gaussian((0, 0, z), (0.5,) * 3, (1, 0, 0, 0), o, rgb) for z, o, rgb in specs]
    r = oracle.render(stack(*gs), cam, px=[8], py=[8])
    al = []
    for z, o, _ in specs:
        var = (cam.fx * 0.5 / z) ** 2 + 0.3
        al.append(min(0.99, o * math.exp(-0.5 * 0.5 / var)))      # pixel centre is 0.5 px off in x and y
    T2 = (1 - al[0]) * (1 - al[1])
    assert T2 > 1e-4 and T2 * (1 - al[2]) < 1e-4 and T2 * (1 - al[3]) > 1e-4
    want = np.array([al[0], al[1] * (1 - al[0]), 0.0]) + T2 * np.array(cam.bg)
    np.testing.assert_allclose(r["image"][0], want, atol=1e-12)
    assert r["nblend"][0] == 2 and r["last_id"][0] == 1
    np.testing.assert_allclose(r["final_T"][0], T2, rtol=1e-12)


def test_compositing_invariants_random_scenes():
    """Pixels are convex combinations of the Gaussian colours and the
    background; final T stays at or above 1e-4."""
    for seed in range(3):
        g, cam, _ = scenes.config1(seed=seed + 10)
        r = oracle.render(g, cam)
        p = oracle.project(g, cam)
        lo = min(p["rgb"].min(), min(cam.bg)) - 1e-12
        hi = max(p["rgb"].max(), max(cam.bg)) + 1e-12
        assert r["image"].min() >= lo and r["image"].max() <= hi
        assert r["final_T"].min() >= 1e-4 and r["final_T"].max() <= 1.0
        # with a white background and colours in [0, 1], 1 - pixel <= 1 - T
        assert np.all(1 - r["image"] <= (1 - r["final_T"])[None] + 1e-12)


# ------------------------------------------------------------- binning --

def _brute_bins(b, cam, tw, th, n):
    ntx = (cam.width + tw - 1) // tw
    pairs = []
    for i in range(n):
        x0, y0, x1, y1 = b["trect"][i]
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                pairs.append(((int(ty * ntx + tx) << 32) | int(b["zbits"][i]), i))
    pairs.sort()
    return pairs


@pytest.mark.parametrize("tw,th", [(16, 16), (8, 8), (32, 8)])
def test_binning_is_a_stable_sort_and_ranges_are_equal_ranges(tw, th):
    g, cam, _ = scenes.config1()
    b = oracle.bin(g, cam, tw, th)
    pairs = _brute_bins(b, cam, tw, th, g.n)
    assert len(pairs) == len(b["keys"])
    assert [k for k, _ in pairs] == [int(k) for k in b["keys"]]
    assert [v for _, v in pairs] == [int(v) for v in b["vals"]]
    tiles = (b["keys"] >> np.uint64(32)).astype(np.int64)
    for t in range(b["ranges"].shape[0]):
        lo, hi = np.searchsorted(tiles, t, "left"), np.searchsorted(tiles, t, "right")
        if lo == hi:
            assert tuple(b["ranges"][t]) == (0, 0)
        else:
            assert tuple(b["ranges"][t]) == (lo, hi)
    # the scan of tiles_touched is the pair count
    assert int(b["tiles_touched"].astype(np.int64).sum()) == len(b["keys"])


def test_tile_rectangles_are_conservative():
    """Every pixel whose alpha reaches 1/255 lies inside its Gaussian's
    pixel rectangle (brute force over the image, high opacities too)."""
    g, cam, _ = scenes.config1(seed=4)
    g.opacity[:] = np.linspace(0.01, 0.999, g.n).astype(np.float32)
    p = oracle.project(g, cam)
    xs, ys = pixel_grid(cam)
    for i in range(0, g.n, 7):
        A, B, Cc = p["conic"][i]
        u, v = p["uv"][i]
        dx, dy = xs - u, ys - v
        a = g.opacity[i] * np.exp(-0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy)
        inside = a >= 1 / 255
        if not p["valid"][i]:
            assert not inside.any()
            continue
        x0, y0, x1, y1 = p["pxrect"][i]
        iy, ix = np.nonzero(inside)
        assert ix.min() >= x0 and ix.max() <= x1 and iy.min() >= y0 and iy.max() <= y1
        # the rectangle is the tight bounding box of the ellipse (clamped)
        assert (ix.min() - x0) <= 1 and (x1 - ix.max()) <= 1


@pytest.mark.parametrize("tw,th", [(16, 16), (8, 8), (32, 32)])
def test_tiled_evaluation_equals_all_pairs(tw, th):
    """Brute force: blending each pixel's tile list gives exactly the plain
    all-pairs image (binning is a pure acceleration)."""
    g, cam, _ = scenes.config1(seed=5)
    g.opacity[::3] = 0.995      # high opacities, where a 3-sigma bound would not be conservative
    full = oracle.render(g, cam)
    b = oracle.bin(g, cam, tw, th)
    img, fT = oracle.render_tiled(g, cam, b["vals"], b["ranges"], tw, th)
    np.testing.assert_array_equal(img, full["image"])
    np.testing.assert_array_equal(fT, full["final_T"])


# ------------------------------------------------------------ gradients --

def _tiny_scene(seed, n=6, deg=3, W=24, H=20):
    rng = np.random.default_rng(seed)
    cam = scenes.look_at((0.3, 0.2, -4.0), (0, 0, 0), W, H, hfov_deg=55, bg=(0.3, 0.5, 0.2))
    K = (deg + 1) ** 2
    mean = np.stack([rng.uniform(-0.6, 0.6, n), rng.uniform(-0.5, 0.5, n), rng.uniform(-0.8, 0.8, n)])
    scale = np.exp(rng.normal(-1.6, 0.3, (3, n)))
    quat = rng.normal(size=(4, n))
    opac = rng.uniform(0.3, 0.8, n)
    sh = rng.normal(0, 0.3, (3 * K, n))
    sh[0::K] = rng.uniform(-0.5, 1.5, (3, n))
    if n > 5:
        sh[K, 2] = -4.0                  # one clamped colour channel
        mean[:, 5] = [3.2, 0.0, 0.3]     # beyond the 1.3x field-of-view clamp, footprint in the image
        scale[:, 5] = [0.9, 0.7, 0.8]
        opac[5] = 0.9
    g = scenes.Gaussians(mean, scale, quat, opac, sh, deg)
    w = rng.normal(size=(3, H, W))
    return g, cam, w


def _loss(g, cam, w):
    return float((oracle.render(g, cam)["image"] * w).sum())


def _signature(g, cam):
    r = oracle.render(g, cam)
    return r["nblend"], r["last_id"]


@pytest.mark.parametrize("seed", [0, 1])
def test_analytic_gradient_matches_central_differences(seed):
    g, cam, w = _tiny_scene(seed)
    an = oracle.backward(g, cam, w)
    # the Gaussian beyond the clamp contributes (its clamped Jacobian is exercised)
    Rm = np.asarray(cam.R, np.float64).reshape(3, 3)
    t5 = Rm @ g.mean[:, 5] + np.asarray(cam.t, np.float64)
    assert abs(t5[0] / t5[2]) > 1.3 * (cam.width / 2) / cam.fx
    assert abs(an["opacity"][5]) > 1e-6 and abs(an["mean"][2, 5]) > 1e-6
    groups = {"mean": g.mean, "scale": g.scale, "quat": g.quat, "opacity": g.opacity, "sh": g.sh}
    sig0 = _signature(g, cam)
    checked = 0
    for name, arr in groups.items():
        flat = arr.reshape(-1)
        gan = an[name].reshape(-1)
        for j in range(flat.size):
            x0 = flat[j]
            h = 1e-6 * max(1.0, abs(x0))
            flat[j] = x0 + h
            lp, sp = _loss(g, cam, w), _signature(g, cam)
            flat[j] = x0 - h
            lm, sm = _loss(g, cam, w), _signature(g, cam)
            flat[j] = x0
            if not all(np.array_equal(a, b) for a, b in zip(sp + sm, sig0 + sig0)):
                continue        # a threshold decision flipped inside +-h
            fd = (lp - lm) / (2 * h)
            assert abs(gan[j] - fd) <= 1e-5 * abs(fd) + 1e-7, (name, j, gan[j], fd)
            checked += 1
    assert checked > 300


def test_gradient_restricted_to_pixel_sample_equals_masked_full_gradient():
    """Listing pixels only restricts the sum: the gradient over a pixel
    list equals the full-frame gradient of a dL/dI that is zero elsewhere."""
    g, cam, w = _tiny_scene(4)
    px, py = scenes.pixel_sample(cam.width, cam.height, stride=5, offset=1)
    m = np.zeros_like(w)
    m[:, py, px] = w[:, py, px]
    full = oracle.backward(g, cam, m)
    part = oracle.backward(g, cam, w * (m != 0), px=px, py=py)
    for k in ("mean", "scale", "quat", "opacity", "sh"):
        np.testing.assert_allclose(part[k], full[k], rtol=1e-12, atol=1e-15)


# -------------------------------------------------- alpha capped at 0.99 --

def _capped_scene(seed, W=40, H=32):
    """Seven Gaussians, three of them with opacity 0.995-0.9999 and wide
    enough that the pixel centres nearest their centres take alpha = 0.99
    (capped) while a wide ring around them does not."""
    rng = np.random.default_rng(seed)
    cam = scenes.look_at((0.2, 0.1, -5.0), (0, 0, 0), W, H, hfov_deg=50, bg=(0.2, 0.4, 0.3))
    n, deg = 7, 1
    K = (deg + 1) ** 2
    mean = np.stack([rng.uniform(-0.7, 0.7, n), rng.uniform(-0.5, 0.5, n), rng.uniform(-0.6, 0.6, n)])
    scale = np.exp(rng.normal(-1.7, 0.3, (3, n)))
    opac = rng.uniform(0.3, 0.8, n)
    opac[:3] = [0.995, 0.999, 0.9999]
    scale[:, :3] = rng.uniform(0.7, 1.1, (3, 3))
    quat = rng.normal(size=(4, n))
    sh = rng.normal(0, 0.3, (3 * K, n))
    sh[0::K] = rng.uniform(-0.5, 1.5, (3, n))
    g = scenes.Gaussians(mean, scale, quat, opac, sh, deg)
    w = rng.normal(size=(3, H, W))
    return g, cam, w


def _capped_contributions(g, cam, i):
    """Pixels where Gaussian i is blended with alpha capped at 0.99, and
    pixels where it is blended below the cap (recomputed here from the
    oracle's own blend order, in plain NumPy)."""
    pr = oracle.project(g, cam)
    r = oracle.render(g, cam)
    W, H = cam.width, cam.height
    ys, xs = np.mgrid[0:H, 0:W]
    u, v = pr["uv"][i]
    A, B, C = pr["conic"][i]
    dx, dy = xs + 0.5 - u, ys + 0.5 - v
    a = g.opacity[i] * np.exp(-0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy)
    order = np.argsort(pr["depth"], kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    # blended at a pixel iff it lies at or before the pixel's last blended Gaussian
    last = r["last_id"]
    reached = (last >= 0) & (rank[np.maximum(last, 0)] >= rank[i])
    return reached & (a > 0.99), reached & (a >= 1 / 255) & (a <= 0.99)


def _fd_mismatches(g, cam, w, names=("mean", "scale", "quat", "opacity")):
    """Central differences (h = 1e-6 relative) of L = sum(w * I) against
    the oracle's analytic gradient, skipping components whose +-h renders
    change a blend decision or come near one (flags, including the 0.99
    cap window).  Returns (mismatches, checked)."""
    w = w * (oracle.render(g, cam)["flags"] == 0)     # no weight on ambiguous pixels
    an = oracle.backward(g, cam, w)
    live = np.abs(w).sum(0) > 0

    def sig(r):
        return r["nblend"][live], r["last_id"][live], r["flags"][live]

    bad, checked = [], 0
    for name in names:
        arr = getattr(g, name)
        flat = arr.reshape(-1)
        gan = an[name].reshape(-1)
        for j in range(flat.size):
            x0 = flat[j]
            h = 1e-6 * max(1.0, abs(x0))
            flat[j] = x0 + h
            rp = oracle.render(g, cam)
            flat[j] = x0 - h
            rm = oracle.render(g, cam)
            flat[j] = x0
            sp, sm = sig(rp), sig(rm)
            if (sp[2] != 0).any() or (sm[2] != 0).any() or \
                    not all(np.array_equal(a, b) for a, b in zip(sp, sm)):
                continue
            fd = float(((rp["image"] - rm["image"]) * w).sum()) / (2 * h)
            checked += 1
            if abs(gan[j] - fd) > 1e-5 * abs(fd) + 1e-7:
                bad.append((name, j, float(gan[j]), fd))
    return bad, checked


@pytest.mark.parametrize("seed", [0, 1])
def test_capped_alpha_gradient_matches_central_differences(seed):
    """Where alpha = min(0.99, o exp(power)) takes the cap, alpha depends on
    neither o nor the geometry: the opacity, mean, scale and rotation
    gradients of Gaussians that are capped at their centre pixels and not
    in the ring around them agree with central differences."""
    g, cam, w = _capped_scene(seed)
    for i in range(3):
        cap, ring = _capped_contributions(g, cam, i)
        assert cap.sum() >= 1 and ring.sum() >= 100, (i, int(cap.sum()), int(ring.sum()))
    bad, checked = _fd_mismatches(g, cam, w)
    assert checked >= 60
    assert not bad, bad[:5]


def test_planted_capped_opacity_gradient_is_caught(tmp_path):
    """A slip that keeps dL/do = dL/dalpha * G under the cap (planted in the
    oracle, on the CPU) fails the central-difference pin above."""
    g, cam, w = _capped_scene(0)
    path = oracle.build_planted("ORC_PLANT_CAPPED_DOPACITY", str(tmp_path))
    with oracle.planted_library(path):
        bad, checked = _fd_mismatches(g, cam, w, names=("opacity",))
    assert checked >= 3
    assert {j for name, j, _, _ in bad} >= {0, 1, 2}, bad
