"""Pins of the FP64 oracle against things other than itself: closed forms,
library routines, invariants and brute force.  CPU only."""
import math

import numpy as np
import pytest

import synth
from synth import Camera, Instance, Scene

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def axis_camera(W=64, H=64, fovy_deg=60.0, near=0.2):
    """Camera at the origin looking along +z with x right and y down."""
    return Camera(pos=np.zeros(3, np.float32), R=np.eye(3, dtype=np.float32),
                  fovy=math.radians(fovy_deg), width=W, height=H, near=near)


def one_gaussian_asset(mean, scale, quat=(1, 0, 0, 0), opacity=0.8, rgb=(0.2, 0.5, 0.9), degree=0):
    n = 1
    a = synth.Asset(mean=np.asarray(mean, np.float32).reshape(3, n),
                    scale=np.asarray(scale, np.float32).reshape(3, n),
                    quat=np.asarray(quat, np.float32).reshape(4, n),
                    opacity=np.asarray([opacity], np.float32),
                    sh=((np.asarray(rgb, np.float64) - 0.5) / (0.5 / math.sqrt(math.pi))).astype(np.float32).reshape(3, n),
                    sh_degree=degree, mlp=synth.MLPSpec(params=synth.mlp_params(8, synth.rng(0)), width=8))
    return a


def project_one(orc, asset, cam, inst=None):
    inst = inst or synth.identity_instance(0)
    sc = Scene(assets=[asset], instances=[inst], cameras=[cam])
    rec, prect = orc.project(sc, cam, np.zeros(1, np.int64))
    return rec[0], prect[0]


# ---------------------------------------------------------------------------
# encoding (Sec. 3.2 counting) and MLP
# ---------------------------------------------------------------------------
def test_encoding_count_matches_paper(orc):
    # the paper counts five bands over the six scalars as sixty values
    assert orc.encode(np.zeros(6), bands=5).size == 60
    assert orc.encode(np.zeros(6), bands=6).size == 72


def test_encoding_angle_doubling(orc):
    x = np.random.default_rng(1).uniform(-1.3, 1.3, 6)
    e = orc.encode(x, bands=6).reshape(6, 6, 2)
    # sin(2a) = 2 sin a cos a, cos(2a) = 1 - 2 sin^2 a, band 0 is sin/cos(pi x)
    np.testing.assert_allclose(e[:, 0, 0], np.sin(np.pi * x), atol=1e-15)
    np.testing.assert_allclose(e[:, 0, 1], np.cos(np.pi * x), atol=1e-15)
    for k in range(5):
        np.testing.assert_allclose(e[:, k + 1, 0], 2 * e[:, k, 0] * e[:, k, 1], atol=1e-12)
        np.testing.assert_allclose(e[:, k + 1, 1], 1 - 2 * e[:, k, 0] ** 2, atol=1e-12)
    z = orc.encode(np.zeros(2), bands=3).reshape(2, 3, 2)
    assert np.all(z[..., 0] == 0) and np.all(z[..., 1] == 1)


def _numpy_mlp(params, W, X):
    off = 0
    h = X
    fan = X.shape[1]
    for _ in range(3):
        Wl = params[off:off + W * fan].reshape(W, fan); off += W * fan
        bl = params[off:off + W]; off += W
        h = np.maximum(h @ Wl.T + bl, 0.0)
        fan = W
    wo = params[off:off + W]; bo = params[off + W]
    return h @ wo + bo


@pytest.mark.parametrize("W", [64, 128])
def test_mlp_equals_numpy_matmul_chain(orc, W):
    g = np.random.default_rng(W)
    p = synth.mlp_params(W, synth.rng(W)).astype(np.float64)
    assert p.size == synth.mlp_param_count(W) == {64: 13057, 128: 42497}[W]
    X = g.uniform(-1, 1, (300, 72))
    z, _ = orc.mlp_forward(p, W, X)
    ref = _numpy_mlp(p, W, X)
    np.testing.assert_allclose(z, ref, rtol=1e-12, atol=1e-12)


def test_mlp_bias_only_is_constant(orc):
    W = 16
    p = synth.mlp_params(W, synth.rng(3)).astype(np.float64)
    n1 = 72 * W
    p[:n1] = 0
    p[n1 + W:n1 + W + W * W] = 0
    o = n1 + W + W * W + W
    p[o:o + W * W] = 0
    b3 = p[o + W * W:o + W * W + W]
    wo = p[-W - 1:-1]
    X = np.random.default_rng(0).uniform(-1, 1, (50, 72))
    z, _ = orc.mlp_forward(p, W, X)
    np.testing.assert_allclose(z, np.dot(wo, np.maximum(b3, 0)) + p[-1], rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# scene transform, Eq. 2 and the frustum
# ---------------------------------------------------------------------------
def test_local_camera_eq2_fov_and_scale(orc):
    inst = Instance(asset=0, R=synth.yaw(0.7), s=2.0, t=np.array([3.0, -1.0, 0.5], np.float32))
    cam = synth.camera((10.0, 4.0, 6.0), fovy_deg=20.0, width=300, height=200)
    f_t = 256.0 / math.tan(math.radians(30.0))  # trained at 60 deg, 512 px tall
    cl = orc.local_camera(inst, cam, f_t)
    d_r = np.linalg.norm(np.asarray(cam.pos, np.float64) - inst.t)
    # Eq. 2: d_t = d_r (f_t / f_r) / s with focal lengths in pixels (H/2) / tan(fovy/2)
    f_r = 100.0 / math.tan(float(np.float32(math.radians(20.0))) / 2)
    d_t = d_r * (f_t / f_r) / 2.0
    # (the float32 rotation is orthonormal to ~1e-7)
    assert abs(np.linalg.norm(cl) - d_t) < 2e-7 * d_t
    # direction: R^T (c - t) / |c - t|
    dir_ = inst.R.astype(np.float64).T @ (np.asarray(cam.pos, np.float64) - inst.t)
    np.testing.assert_allclose(cl / np.linalg.norm(cl), dir_ / np.linalg.norm(dir_), atol=1e-12)
    # same resolution, FoV 60 -> 20: the distance shrinks by tan 10 / tan 30
    cam2 = synth.camera((10.0, 4.0, 6.0), fovy_deg=20.0, width=512, height=512)
    cl2 = orc.local_camera(inst, cam2, f_t)
    ratio = np.linalg.norm(cl2) * 2.0 / d_r
    assert abs(ratio - math.tan(float(np.float32(math.radians(20.0))) / 2) / math.tan(math.radians(30))) < 2e-7
    # same FoV, twice the resolution: half the distance
    cam3 = synth.camera((10.0, 4.0, 6.0), fovy_deg=60.0, width=1024, height=1024)
    cl3 = orc.local_camera(inst, cam3, f_t)
    assert abs(np.linalg.norm(cl3) * 2.0 / d_r - 0.5) < 2e-7
    # the far clamp keeps the direction and caps the length
    clc = orc.local_camera(inst, cam, f_t, d_max=0.5 * d_t)
    assert abs(np.linalg.norm(clc) - 0.5 * d_t) < 1e-12
    np.testing.assert_allclose(clc / np.linalg.norm(clc), dir_ / np.linalg.norm(dir_), atol=1e-12)


def test_eq1_distance_range():
    # Eq. 1: d = r / (tan(theta/2) p) for the torus (half-diagonal 1.941) at 50 deg
    r = synth.SHAPE_HALF_DIAG["torus"]
    assert abs(r - 1.9411) < 1e-3
    d_near = r / (math.tan(math.radians(25)) * 0.9)
    d_far = r / (math.tan(math.radians(25)) * 0.05)
    assert abs(d_near - 4.625) < 5e-3 and abs(d_far - 83.25) < 0.1


def test_frustum_special_points(orc):
    cam = axis_camera(W=64, H=32, fovy_deg=60.0)
    ty = math.tan(math.radians(30))
    tx = ty * 2.0
    pts = {
        (0.0, 0.0, 1.0): 2,              # on the axis
        (0.0, 0.0, 0.1): 0,              # before the near plane
        (0.0, 0.0, 0.2): 0,              # exactly at near: p_z > near is strict
        (1.29 * tx * 5, 0.0, 5.0): 2,    # inside the 1.3 guard band in x
        (1.31 * tx * 5, 0.0, 5.0): 0,
        (0.0, -1.29 * ty * 5, 5.0): 2,
        (0.0, 1.31 * ty * 5, 5.0): 0,
        (0.0, 0.0, -3.0): 0,             # behind
        (0.0, 0.0, 1e6): 2,              # no far plane
    }
    means = np.array(list(pts.keys()), np.float32).T.copy()
    a = synth.Asset(mean=means, scale=np.ones_like(means) * 0.01, quat=np.tile([[1], [0], [0], [0]], means.shape[1]).astype(np.float32),
                    opacity=np.ones(means.shape[1], np.float32), sh=np.zeros((3, means.shape[1]), np.float32),
                    sh_degree=0, mlp=synth.MLPSpec(params=synth.mlp_params(8, synth.rng(0)), width=8))
    sc = Scene(assets=[a], instances=[synth.identity_instance()], cameras=[cam])
    st, lg = orc.query(sc, use_mlp=False)
    assert st[0].tolist() == list(pts.values())
    assert np.all(np.isnan(lg))


def _random_scene(n=3000, seed=5, W=48, H=40, degree=3, width=16):
    a = synth.make_asset("torus", n, degree, seed, width=width)
    inst = Instance(asset=0, R=synth.yaw(1.1) @ np.array([[1, 0, 0], [0, 0.6, -0.8], [0, 0.8, 0.6]], np.float32),
                    s=1.7, t=np.array([0.4, -0.3, 0.2], np.float32))
    cam = synth.camera((0.5, -5.0, 2.5), target=(0.4, -0.3, 0.2), fovy_deg=45.0, width=W, height=H)
    return Scene(assets=[a], instances=[inst], cameras=[cam], tile=8)


def _mapped_identity_scene(sc):
    """The same view with an identity instance and the camera mapped by the
    inverse instance transform (near plane scaled with it)."""
    inst, cam = sc.instances[0], sc.cameras[0]
    R = inst.R.astype(np.float64)
    pos = R.T @ (np.asarray(cam.pos, np.float64) - inst.t) / inst.s
    cam2 = Camera(pos=pos, R=cam.R.astype(np.float64) @ R, fovy=cam.fovy, width=cam.width,
                  height=cam.height, near=cam.near / inst.s)
    return Scene(assets=sc.assets, instances=[synth.identity_instance()], cameras=[cam2], tile=sc.tile)


@pytest.mark.parametrize("exact", [True, False])
def test_instancing_invariance(orc, exact):
    sc = _random_scene()
    tol = 1e-9
    if exact:
        # signed-permutation rotation, power-of-two scale and dyadic offsets:
        # the inverse-mapped camera is exactly representable in float32
        sc.instances[0] = Instance(asset=0, R=np.array([[0, 0, 1], [-1, 0, 0], [0, -1, 0]], np.float32),
                                   s=2.0, t=np.array([0.5, -0.25, 0.125], np.float32))
        sc.cameras[0] = Camera(pos=np.array([1.0, -6.0, 3.0], np.float32),
                               R=np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], np.float32),
                               fovy=sc.cameras[0].fovy, width=48, height=40, near=0.25)
    else:
        tol = 1e-5  # float32 rounding of the mapped camera
    sc2 = _mapped_identity_scene(sc)
    st1, lg1 = orc.query(sc)
    st2, lg2 = orc.query(sc2)
    assert np.array_equal(st1, st2)
    q = ~np.isnan(lg1)
    assert q.sum() > 100 and np.array_equal(q, ~np.isnan(lg2))
    np.testing.assert_allclose(lg1[q], lg2[q], rtol=tol, atol=tol)
    f1 = orc.frame(sc)
    f2 = orc.frame(sc2)
    r1, r2 = f1["rec"][0], f2["rec"][0]
    np.testing.assert_allclose(r1[:, [0, 1, 2, 3, 4, 9, 10, 11, 12]], r2[:, [0, 1, 2, 3, 4, 9, 10, 11, 12]],
                               rtol=tol, atol=tol)
    np.testing.assert_allclose(r1[:, 8], r2[:, 8] * sc.instances[0].s, rtol=tol)
    np.testing.assert_allclose(f1["images"][0], f2["images"][0], atol=100 * tol)


# ---------------------------------------------------------------------------
# EWA projection closed forms
# ---------------------------------------------------------------------------
def test_projection_on_axis_closed_form(orc):
    cam = axis_camera(W=64, H=48, fovy_deg=60.0)
    f = 0.5 * 48 / math.tan(float(np.float32(math.radians(60))) / 2)
    z, sx, sy, sz = 4.0, *map(float, np.float32([0.05, 0.11, 0.3]))
    rec, _ = project_one(orc, one_gaussian_asset((0, 0, z), (sx, sy, sz)), cam)
    assert abs(rec[0] - 32.0) < 1e-12 and abs(rec[1] - 24.0) < 1e-12 and rec[8] == z
    assert abs(rec[2] - (f * f * sx * sx / z ** 2 + 0.3)) < 1e-12
    assert abs(rec[4] - (f * f * sy * sy / z ** 2 + 0.3)) < 1e-12
    assert abs(rec[3]) < 1e-15
    # conic is the inverse of Sigma2D
    S = np.array([[rec[2], rec[3]], [rec[3], rec[4]]])
    Ci = np.array([[rec[5], rec[6]], [rec[6], rec[7]]])
    np.testing.assert_allclose(S @ Ci, np.eye(2), atol=1e-12)


def test_projection_off_axis_closed_form(orc):
    cam = axis_camera(W=64, H=48, fovy_deg=60.0)
    f = 0.5 * 48 / math.tan(float(np.float32(math.radians(60))) / 2)
    tx, z, sx, sy, sz = 1.25, 5.0, *map(float, np.float32([0.07, 0.02, 0.2]))
    rec, _ = project_one(orc, one_gaussian_asset((tx, 0, z), (sx, sy, sz)), cam)
    assert abs(rec[2] - (f * f * (sx * sx / z ** 2 + tx * tx * sz * sz / z ** 4) + 0.3)) < 1e-11
    assert abs(rec[3]) < 1e-15
    assert abs(rec[4] - (f * f * sy * sy / z ** 2 + 0.3)) < 1e-11
    assert abs(rec[0] - (f * tx / z + 32.0)) < 1e-12
    # off-axis in both x and y: the depth variance couples u and v
    ty = -0.75
    rec, _ = project_one(orc, one_gaussian_asset((tx, ty, z), (sx, sy, sz)), cam)
    assert abs(rec[3] - f * f * tx * ty * sz * sz / z ** 4) < 1e-11
    assert abs(rec[4] - (f * f * (sy * sy / z ** 2 + ty * ty * sz * sz / z ** 4) + 0.3)) < 1e-11


def test_projection_is_first_order_pushforward(orc):
    """EWA: Sigma2D - 0.3 I = J Sigma_c J^T with J the derivative of the
    perspective map (u, v)(p) at the mean; J is taken here by central
    differences of the map itself, for a rotated, off-axis Gaussian under a
    rotated, scaled instance and a tilted camera."""
    cam = synth.camera((0.3, -4.0, 1.5), target=(0.5, 0.2, 0.1), fovy_deg=55.0, width=80, height=60)
    inst = Instance(asset=0, R=synth.yaw(0.4), s=1.5, t=np.array([0.2, 0.1, -0.1], np.float32))
    q = np.array([0.8, 0.3, -0.4, 0.34], np.float64); q /= np.linalg.norm(q)
    a = one_gaussian_asset((0.6, 0.4, 0.3), (0.3, 0.05, 0.12), quat=q)
    rec, _ = project_one(orc, a, cam, inst)
    ca = orc.cam_array(cam); ia = orc.inst_array(inst)
    Rc = ca[3:12].reshape(3, 3); pos = ca[:3]; Ri = ia[:9].reshape(3, 3); s = ia[9]; t = ia[10:13]
    f = 0.5 * 60 / math.tan(0.5 * ca[12])
    uv = lambda pp: np.array([f * pp[0] / pp[2] + 40, f * pp[1] / pp[2] + 30])
    mu = a.mean[:, 0].astype(np.float64)
    p = Rc @ (s * Ri @ mu + t - pos)
    h = 1e-5
    J = np.stack([(uv(p + h * e) - uv(p - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
    qq = a.quat[:, 0].astype(np.float64); qq /= np.linalg.norm(qq)
    w, x, y, z = qq
    Rq = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                   [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                   [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
    # the rotation maps the first scale axis onto its first column
    Sl = Rq @ np.diag(a.scale[:, 0].astype(np.float64) ** 2) @ Rq.T
    M = Rc @ Ri
    Sc = s * s * M @ Sl @ M.T
    S2 = J @ Sc @ J.T
    np.testing.assert_allclose([rec[2] - 0.3, rec[3], rec[4] - 0.3], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-7)
    np.testing.assert_allclose(rec[:2], uv(p), rtol=1e-12)


def test_quaternion_orientation(orc):
    # 30 deg about the view axis turns the long axis towards +x+y: the screen
    # covariance xy term is positive and equals (s1^2 - s2^2) cos30 sin30 f^2/z^2
    cam = axis_camera(64, 64, fovy_deg=60.0)
    f = 0.5 * 64 / math.tan(float(np.float32(math.radians(60))) / 2)
    c, sn = math.cos(math.radians(15)), math.sin(math.radians(15))
    s1, s2 = map(float, np.float32([0.2, 0.02]))
    rec, _ = project_one(orc, one_gaussian_asset((0, 0, 4.0), (s1, s2, 0.02), quat=(c, 0, 0, sn)), cam)
    expect = (s1 * s1 - s2 * s2) * math.cos(math.radians(30)) * math.sin(math.radians(30)) * f * f / 16.0
    assert rec[3] > 0 and abs(rec[3] - expect) < 1e-6 * expect


def test_sh_view_direction_is_camera_to_gaussian(orc):
    # only the (l=1, m=0) coefficient is set: colour = 0.5 + c Y_10(d) with d
    # the unit vector from the camera to the Gaussian in the asset frame
    cam = axis_camera(32, 32)  # at the origin looking along +z
    a = one_gaussian_asset((0, 0, 3.0), (0.05, 0.05, 0.05))
    a.sh_degree = 1
    a.sh = np.zeros((12, 1), np.float32)
    a.sh[3 * 2 + 0, 0] = 0.4  # coefficient 2 = (l=1, m=0), red channel
    rec, _ = project_one(orc, a, cam)
    y10 = math.sqrt(3 / (4 * math.pi))
    assert abs(rec[10] - (0.5 + 0.4 * y10)) < 1e-7 and abs(rec[11] - 0.5) < 1e-12


def test_projection_rotation_about_view_axis_swaps(orc):
    cam = axis_camera()
    a = one_gaussian_asset((0, 0, 3.0), (0.09, 0.03, 0.05))
    r0, _ = project_one(orc, a, cam)
    h = math.sqrt(0.5)
    b = one_gaussian_asset((0, 0, 3.0), (0.09, 0.03, 0.05), quat=(h, 0, 0, h))  # 90 deg about z
    r1, _ = project_one(orc, b, cam)
    assert abs(r0[2] - r1[4]) < 1e-12 and abs(r0[4] - r1[2]) < 1e-12
    # an unnormalised quaternion is normalised on use
    c = one_gaussian_asset((0, 0, 3.0), (0.09, 0.03, 0.05), quat=(3 * h, 0, 0, 3 * h))
    r2, _ = project_one(orc, c, cam)
    np.testing.assert_allclose(r1, r2, atol=1e-12)


# ---------------------------------------------------------------------------
# spherical harmonics
# ---------------------------------------------------------------------------
def _real_sh_scipy(l, m, theta, phi):
    from scipy import special
    try:
        Y = lambda mm: special.sph_harm_y(l, mm, theta, phi)
    except AttributeError:  # older scipy
        Y = lambda mm: special.sph_harm(mm, l, phi, theta)
    if m == 0:
        return Y(0).real
    # real form without Condon-Shortley phase: the (-1)^m cancels scipy's phase
    if m > 0:
        return math.sqrt(2) * (-1) ** m * Y(m).real
    return math.sqrt(2) * (-1) ** m * Y(-m).imag


def test_sh_basis_matches_scipy_real_form(orc):
    g = np.random.default_rng(2)
    for _ in range(20):
        d = g.standard_normal(3)
        d /= np.linalg.norm(d)
        theta = math.acos(d[2])
        phi = math.atan2(d[1], d[0])
        Y = orc.sh_basis(d, 3)
        k = 0
        for l in range(4):
            for m in range(-l, l + 1):
                assert abs(Y[k] - _real_sh_scipy(l, m, theta, phi)) < 1e-12, (l, m)
                k += 1


def test_sh_orthonormal_by_quadrature(orc):
    # Gauss-Legendre in cos(theta) x uniform phi integrates degree <= 6 exactly
    xs, ws = np.polynomial.legendre.leggauss(12)
    nphi = 16
    G = np.zeros((16, 16))
    for x, w in zip(xs, ws):
        st = math.sqrt(1 - x * x)
        for j in range(nphi):
            ph = 2 * math.pi * j / nphi
            Y = orc.sh_basis(np.array([st * math.cos(ph), st * math.sin(ph), x]), 3)
            G += w * (2 * math.pi / nphi) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh0_colour_is_sampled_rgb(orc):
    cam = axis_camera()
    a = one_gaussian_asset((0.1, -0.2, 3.0), (0.05, 0.05, 0.05), rgb=(0.25, 0.5, 0.75))
    rec, _ = project_one(orc, a, cam)
    np.testing.assert_allclose(rec[10:13], [0.25, 0.5, 0.75], atol=1e-7)


# ---------------------------------------------------------------------------
# compositing
# ---------------------------------------------------------------------------
def _rec(u, v, sxx, sxy, syy, depth, o, rgb):
    det = sxx * syy - sxy * sxy
    r = np.zeros(16)
    r[0], r[1], r[2], r[3], r[4] = u, v, sxx, sxy, syy
    r[5], r[6], r[7] = syy / det, -sxy / det, sxx / det
    r[8], r[9] = depth, o
    r[10:13] = rgb
    return r


def _full_rect(m, W, H):
    return np.tile(np.array([[0, W - 1, 0, H - 1]], np.int32), (m, 1))


def test_single_splat_alpha_falloff(orc):
    W = H = 16
    cam = axis_camera(W, H)
    for o in (0.5, 1.0):
        rec = _rec(7.5, 8.5, 4.0, 0.0, 1.0, 2.0, o, (0.3, 0.6, 0.9))[None]
        out = orc.render_camera(rec, _full_rect(1, W, H), cam, 16)
        img = out["image"]
        a0 = min(0.99, o)
        np.testing.assert_allclose(img[8, 7], a0 * np.array([0.3, 0.6, 0.9]), rtol=1e-14)
        # one sigma along the major (x) axis: dx = 2 -> alpha = o e^(-1/2)
        a1 = min(0.99, o * math.exp(-0.5))
        np.testing.assert_allclose(img[8, 9], a1 * np.array([0.3, 0.6, 0.9]), rtol=1e-14)
        # outside the kappa ellipse nothing is blended
        k2 = 2 * math.log(255 * o)
        for px in range(W):
            q = (px + 0.5 - 7.5) ** 2 / 4.0
            if q > k2 + 1e-9:
                assert np.all(img[8, px] == 0)


def test_two_splat_closed_form(orc):
    cam = axis_camera(8, 8)
    c1, c2 = np.array([1.0, 0.2, 0.1]), np.array([0.1, 0.3, 1.0])
    rec = np.stack([_rec(3.5, 3.5, 1e4, 0, 1e4, 1.0, 0.6, c1), _rec(3.5, 3.5, 1e4, 0, 1e4, 2.0, 0.7, c2)])
    img = orc.render_camera(rec, _full_rect(2, 8, 8), cam, 8, bg=(0.0, 0.0, 0.0))["image"]
    a1, a2 = 0.6, 0.7
    np.testing.assert_allclose(img[3, 3], a1 * c1 + (1 - a1) * a2 * c2, rtol=1e-12)
    # order is by depth, not by id
    rec2 = rec[::-1].copy()
    img2 = orc.render_camera(rec2, _full_rect(2, 8, 8), cam, 8)["image"]
    np.testing.assert_allclose(img2[3, 3], img[3, 3], rtol=1e-14)
    # equal depths: ties break by id
    rec3 = rec.copy(); rec3[1, 8] = 1.0
    img3 = orc.render_camera(rec3, _full_rect(2, 8, 8), cam, 8)["image"]
    np.testing.assert_allclose(img3[3, 3], a1 * c1 + (1 - a1) * a2 * c2, rtol=1e-12)


def test_stop_rule_three_opaque_splats(orc):
    cam = axis_camera(4, 4)
    recs = [_rec(1.5, 1.5, 1e6, 0, 1e6, 1.0 + k, 1.0, (1.0, 1.0, 1.0)) for k in range(4)]
    rec = np.stack(recs)
    cb = np.zeros(4)
    rc = np.zeros(4, np.uint8)
    out = orc.render_camera(rec, _full_rect(4, 4, 4), cam, 4, contrib=cb, reached=rc)
    T = out["T"][1, 1]
    # two splats of alpha 0.99 bring T to 1e-4 (not below): both blended;
    # the third would push T below 1e-4 and is not blended; the fourth is never reached
    assert abs(T - 0.01 * 0.01) < 1e-15 and T >= 1e-4
    assert abs(out["image"][1, 1, 0] - (0.99 + 0.01 * 0.99)) < 1e-14
    assert rc.tolist() == [1, 1, 1, 0]
    assert cb[2] == 0 and cb[3] == 0 and abs(cb[1] - 0.99 * 0.01) < 1e-15


def test_partition_of_unity_and_T_bounds(orc):
    sc = _random_scene(n=4000, degree=0)
    st, _ = orc.query(sc, use_mlp=False)
    kept = orc.compact(st)[0]
    rec, prect = orc.project(sc, sc.cameras[0], kept)
    rec[:, 10:13] = 1.0  # white splats, black background: C + T_final = 1
    out = orc.render_camera(rec, prect, sc.cameras[0], 8)
    np.testing.assert_allclose(out["image"][..., 0] + out["T"], 1.0, atol=1e-12)
    assert np.all(out["T"] >= 1e-4) and np.all(out["T"] <= 1.0)
    assert np.any(out["T"] < 0.5)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_tiled_equals_tile_free_bruteforce(orc, tile):
    sc = _random_scene(n=200, seed=9, W=32, H=32)
    sc.instances[0].s = 3.0
    st, _ = orc.query(sc, use_mlp=False)
    kept = orc.compact(st)[0]
    assert 50 < len(kept) <= 200
    rec, prect = orc.project(sc, sc.cameras[0], kept)
    tiled = orc.render_camera(rec, prect, sc.cameras[0], tile)
    brute, tf = orc.render_brute(rec, sc.cameras[0])
    assert np.array_equal(tiled["image"], brute)
    assert np.array_equal(tiled["T"], tf)


def test_footprint_is_conservative(orc):
    sc = _random_scene(n=400, seed=13, W=40, H=32)
    sc.instances[0].s = 4.0
    st, _ = orc.query(sc, use_mlp=False)
    kept = orc.compact(st)[0]
    rec, prect = orc.project(sc, sc.cameras[0], kept)
    W, H = 40, 32
    px, py = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    for r, pr in zip(rec, prect):
        dx, dy = px - r[0], py - r[1]
        q = r[5] * dx * dx + 2 * r[6] * dx * dy + r[7] * dy * dy
        alpha = np.minimum(0.99, r[9] * np.exp(-0.5 * q))
        ys, xs = np.nonzero(alpha >= 1 / 255)
        if len(xs):
            assert pr[0] <= xs.min() and xs.max() <= pr[1] and pr[2] <= ys.min() and ys.max() <= pr[3]


def test_sort_order_is_tile_depth_id(orc):
    sc = _random_scene(n=500, seed=21, W=48, H=40)
    sc.instances[0].s = 2.5
    st, _ = orc.query(sc, use_mlp=False)
    kept = orc.compact(st)[0]
    rec, prect = orc.project(sc, sc.cameras[0], kept)
    rec[::7, 8] = rec[1, 8]  # force depth ties
    out = orc.render_camera(rec, prect, sc.cameras[0], 8, want_order=True)
    tw = (48 + 7) // 8
    ent = []
    for j, pr in enumerate(prect):
        if pr[0] > pr[1]:
            continue
        for ty in range(pr[2] // 8, pr[3] // 8 + 1):
            for tx in range(pr[0] // 8, pr[1] // 8 + 1):
                ent.append((ty * tw + tx, rec[j, 8], j))
    ref = sorted(ent)
    assert [(t, j) for t, _, j in ref] == [tuple(x) for x in out["order"].tolist()]


def test_ground_truth_visibility_invariant(orc):
    sc = _random_scene(n=6000, seed=31, W=48, H=40, degree=3)
    sc.instances[0].s = 2.0
    f = orc.frame(sc, use_mlp=False, record=True)
    rec, prect = f["rec"][0], f["prect"][0]
    reached, contrib = f["reached"][0], f["contrib"][0]
    assert 0 < reached.sum() < len(reached)
    img = f["images"][0]
    keep = reached == 1
    img2 = orc.render_camera(rec[keep], prect[keep], sc.cameras[0], 8)["image"]
    assert np.array_equal(img, img2)  # removing never-reached splats changes nothing
    keep = contrib > 0
    img3 = orc.render_camera(rec[keep], prect[keep], sc.cameras[0], 8)["image"]
    # removing never-blended splats changes no pixel by more than T_min * max colour
    assert np.max(np.abs(img3 - img)) <= 1e-4 * max(1.0, rec[:, 10:13].max())


def test_labels_on_a_stack(orc):
    # 3 layers of wide opaque splats in front of a layer of small ones: the
    # small ones behind saturated pixels never contribute.
    n_front, n_back = 3, 40
    g = np.random.default_rng(4)
    back = np.stack([g.uniform(-0.3, 0.3, n_back), g.uniform(-0.3, 0.3, n_back), np.full(n_back, 5.0)])
    front = np.stack([np.zeros(n_front), np.zeros(n_front), 2.0 + 0.1 * np.arange(n_front)])
    side = np.array([[3.0], [0.0], [5.0]])  # visible, off to the side
    means = np.concatenate([front, back, side], axis=1).astype(np.float32)
    n = means.shape[1]
    scale = np.full((3, n), 0.01, np.float32)
    scale[:, :n_front] = 1.0
    quat = np.tile([[1], [0], [0], [0]], n).astype(np.float32)
    op = np.full(n, 0.8, np.float32)
    op[:n_front] = 1.0
    a = synth.Asset(mean=means, scale=scale, quat=quat, opacity=op, sh=np.zeros((3, n), np.float32),
                    sh_degree=0, mlp=synth.MLPSpec(params=synth.mlp_params(8, synth.rng(0)), width=8))
    cam = axis_camera(64, 64, fovy_deg=90.0)
    lab = orc.labels(a, [cam])[0]
    assert lab[:n_front].tolist() == [1, 1, 1]  # the front layers contribute
    assert np.all(lab[n_front:n_front + n_back] == 0)
    assert lab[-1] == 1


# ---------------------------------------------------------------------------
# loss, backward, Adam, RNG, metrics
# ---------------------------------------------------------------------------
def test_backward_matches_central_differences_all_params(orc):
    W = 8
    g = np.random.default_rng(7)
    p = synth.mlp_params(W, synth.rng(11)).astype(np.float64)
    X = g.uniform(-1, 1, (64, 72))
    y = (g.uniform(0, 1, 64) > 0.5).astype(np.float64)
    loss, dP, dX = orc.bce_backward(p, W, X, y, want_dx=True)
    eps = 1e-3
    fd = np.zeros_like(p)
    for k in range(p.size):
        pp = p.copy(); pp[k] += eps
        pm = p.copy(); pm[k] -= eps
        fd[k] = (orc.bce_backward(pp, W, X, y)[0] - orc.bce_backward(pm, W, X, y)[0]) / (2 * eps)
    # a central difference across a ReLU kink is not the derivative: leave out
    # the parameters whose +-eps step flips any hidden unit of any sample
    _, _, pre0 = orc.mlp_forward(p, W, X, want_pre=True)
    smooth = np.ones(p.size, bool)
    for k in range(p.size):
        for sgn in (1, -1):
            pp = p.copy(); pp[k] += sgn * eps
            if np.any((orc.mlp_forward(pp, W, X, want_pre=True)[2] > 0) != (pre0 > 0)):
                smooth[k] = False
    assert smooth.mean() > 0.9
    floor = 1e-6 * np.max(np.abs(fd))
    rel = np.abs(dP - fd) / np.maximum(np.abs(fd), floor)
    assert np.linalg.norm((dP - fd)[smooth]) <= 1e-3 * np.linalg.norm(fd[smooth])
    assert np.all(rel[smooth] < 1e-3)
    # input gradient
    k = 5
    Xp = X.copy(); Xp[3, k] += eps
    Xm = X.copy(); Xm[3, k] -= eps
    fdx = (orc.bce_backward(p, W, Xp, y)[0] - orc.bce_backward(p, W, Xm, y)[0]) / (2 * eps)
    assert abs(dX[3, k] - fdx) <= 1e-3 * abs(fdx) + 1e-9
    # the loss itself: mean of max(z,0) - z y + log(1 + e^-|z|)
    z, _ = orc.mlp_forward(p, W, X)
    ref = np.mean(np.logaddexp(0, z) - z * y)
    assert abs(loss - ref) < 1e-12


def test_adam_one_step_closed_form(orc):
    for gval in (0.3, -2.0):
        p = np.array([1.5]); m = np.zeros(1); v = np.zeros(1)
        orc.adam_step(p, np.array([gval]), m, v, 1, lr=1e-3)
        assert abs(p[0] - (1.5 - 1e-3 * gval / (abs(gval) + 1e-8))) < 1e-15
    # second step with the same gradient: m_hat = g, v_hat = g^2 again
    p = np.array([0.0]); m = np.zeros(1); v = np.zeros(1)
    orc.adam_step(p, np.array([0.5]), m, v, 1)
    orc.adam_step(p, np.array([0.5]), m, v, 2)
    assert abs(p[0] + 2e-3 * 0.5 / (0.5 + 1e-8)) < 1e-15


def test_splitmix64_published_values(orc):
    # first outputs of SplitMix64 seeded with 0 and with 1234567
    assert orc.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert orc.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert orc.splitmix64(1234567, 0) == 6457827717110365317
    assert orc.splitmix64(1234567, 1) == 3203168211198807973


def test_psnr(orc):
    a = np.random.default_rng(0).uniform(0, 1, (8, 8, 3))
    assert orc.psnr(a, a) == 100.0
    assert abs(orc.psnr(a, a + 0.01) - 40.0) < 1e-9


def test_aux_views_lie_on_the_cone_and_keep_framing(orc):
    """Auxiliary views (Sec. 3.1): same distance, at the cone angle from the
    main direction, evenly spaced around it, orthonormal orientation, and the
    asset centre stays where the main view sees it."""
    main = synth.camera((1.0, -3.0, 2.0), target=(0.2, 0.1, -0.1), width=64, height=48)
    ang = math.radians(5.0)
    aux = orc.aux_views(main, 6, ang)
    p0 = main.pos.astype(np.float64)
    d = p0 / np.linalg.norm(p0)
    ring = []
    for cam in aux:
        p = cam.pos.astype(np.float64)
        assert abs(np.linalg.norm(p) - np.linalg.norm(p0)) < 1e-5
        assert abs(math.acos(np.clip(np.dot(p, d) / np.linalg.norm(p), -1, 1)) - ang) < 1e-5
        R = cam.R.astype(np.float64)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-6)
        # the centre (origin) in camera coordinates is unchanged by a rigid turn about it
        assert np.allclose(R @ (-p), main.R.astype(np.float64) @ (-p0), atol=1e-5)
        ring.append(p - np.dot(p, d) * d)
    gaps = [np.linalg.norm(ring[j] - ring[(j + 1) % 6]) for j in range(6)]
    assert max(gaps) - min(gaps) < 1e-5
    # zero angle: the auxiliary views coincide with the main view
    for cam in orc.aux_views(main, 3, 0.0):
        assert np.allclose(cam.pos, main.pos) and np.allclose(cam.R, main.R)


def test_labels_with_aux_views_are_a_superset(orc):
    a = synth.make_asset("sphere", 600, 0, 4242, width=16)
    views = synth.label_views(2, seed=11, d_lo=2.0, d_hi=3.0, res=48)
    base = orc.labels(a, views)
    wide = orc.labels(a, views, aux=4, aux_angle=math.radians(10.0))
    assert np.all(wide >= base)
    assert wide.sum() > base.sum()


def test_radius_clipping_by_covariance_determinant(orc):
    """Radius clipping (Sec. 4.3 ablation): a splat is dropped exactly when
    the determinant of its dilated 2D covariance, (f^2 sx^2/z^2 + 0.3)
    (f^2 sy^2/z^2 + 0.3) on the axis, is below the threshold; the image then
    equals the tile-free brute-force render of the scene without it."""
    cam = axis_camera(W=64, H=48, fovy_deg=60.0)
    f = 0.5 * 48 / math.tan(float(np.float32(math.radians(60))) / 2)
    z = 4.0
    small = tuple(map(float, np.float32([0.004, 0.005, 0.01])))
    big = tuple(map(float, np.float32([0.08, 0.06, 0.1])))
    d_small = (f * f * small[0] ** 2 / z ** 2 + 0.3) * (f * f * small[1] ** 2 / z ** 2 + 0.3)
    zb = z - 0.5
    d_big = (f * f * big[0] ** 2 / zb ** 2 + 0.3) * (f * f * big[1] ** 2 / zb ** 2 + 0.3)
    assert d_small < d_big
    tau = math.sqrt(d_small * d_big)  # between the two
    a = one_gaussian_asset((0, 0, z), small)
    b = one_gaussian_asset((0, 0, zb), big, rgb=(0.9, 0.1, 0.1))  # in front of a, on the axis
    for asset, d in ((a, d_small), (b, d_big)):
        sc = Scene(assets=[asset], instances=[synth.identity_instance(0)], cameras=[cam])
        rec, pr = orc.project(sc, cam, np.zeros(1, np.int64), det_clip=tau)
        assert abs(rec[0, 2] * rec[0, 4] - rec[0, 3] ** 2 - d) < 1e-9 * d
        assert (pr[0, 0] > pr[0, 1]) == (d < tau)
        rec0, pr0 = orc.project(sc, cam, np.zeros(1, np.int64))
        assert pr0[0, 0] <= pr0[0, 1]  # visible without clipping
    # two-splat scene: clipped render == brute force of the big splat alone
    both = synth.Asset(mean=np.concatenate([a.mean, b.mean], 1), scale=np.concatenate([a.scale, b.scale], 1),
                       quat=np.concatenate([a.quat, b.quat], 1), opacity=np.concatenate([a.opacity, b.opacity]),
                       sh=np.concatenate([a.sh, b.sh], 1), sh_degree=0, mlp=a.mlp)
    sc2 = Scene(assets=[both], instances=[synth.identity_instance(0)], cameras=[cam])
    rec2, pr2 = orc.project(sc2, cam, np.arange(2), det_clip=tau)
    img = orc.render_camera(rec2, pr2, cam, 8, want_margin=False)["image"]
    scb = Scene(assets=[b], instances=[synth.identity_instance(0)], cameras=[cam])
    recb, prb = orc.project(scb, cam, np.zeros(1, np.int64))
    ref, _ = orc.render_brute(recb, cam)
    assert np.array_equal(img, ref)
    full = orc.render_camera(*orc.project(sc2, cam, np.arange(2)), cam, 8, want_margin=False)["image"]
    assert not np.array_equal(full, img)


# ---------------------------------------------------------------------------
# the compact MLP form (Sec. 3.2, 3.3, 4.1)
# ---------------------------------------------------------------------------
def _np_compact(P, X, XE=None):
    """The two compact MLPs written out with NumPy matmuls."""
    P = np.asarray(P, np.float64)
    o = 0
    def take(r, c):
        nonlocal o
        W = P[o:o + r * c].reshape(r, c); o += r * c
        b = P[o:o + r]; o += r
        return W, b
    W1, b1 = take(32, 16); W2, b2 = take(32, 32); wo, bo = take(1, 32)
    E1, e1 = take(32, 8); E2, e2 = take(32, 32); E3, e3 = take(6, 32)
    relu = lambda a: np.maximum(a, 0)
    if XE is not None:
        emb = relu(relu(XE @ E1.T + e1) @ E2.T + e2) @ E3.T + e3
        X = np.concatenate([X[:, :10], emb], 1)
    return (relu(relu(X @ W1.T + b1) @ W2.T + b2) @ wo.T + bo)[:, 0]


def test_compact_mlps_equal_numpy_chain(orc):
    g = np.random.default_rng(3)
    P = synth.compact_params(g).astype(np.float64)
    assert P.size == synth.COMPACT_VIS_PARAMS + synth.COMPACT_EMB_PARAMS == 3175
    X = g.uniform(-1, 1, (64, 16))
    z, _ = orc.cmlp_forward(P, X)
    np.testing.assert_allclose(z, _np_compact(P, X), rtol=1e-12, atol=1e-12)
    a = one_gaussian_asset((0.1, 0.2, 0.3), (0.02, 0.03, 0.05), quat=(0.3, -0.5, 0.2, 0.7), opacity=0.6)
    a.mlp = synth.MLPSpec(params=P.astype(np.float32), width=32, bands=0, kind=1)
    E, XE = orc.cembed(a)
    Pf = a.mlp.params.astype(np.float64)
    emb_ref = _np_compact(Pf, np.zeros((1, 16)), XE)  # visibility of [0, E]: checks E through a second path
    x = np.concatenate([np.zeros(10), E[0]])[None]
    np.testing.assert_allclose(orc.cmlp_forward(Pf, x)[0], emb_ref, rtol=1e-12, atol=1e-12)
    # the joint model on raw inputs against the NumPy chain through both networks
    XV = g.uniform(-1, 1, (40, 10))
    XE = np.concatenate([g.uniform(0.1, 1, (40, 1)), g.normal(-4.5, 0.3, (40, 3)), g.standard_normal((40, 4))], 1)
    zj, _ = orc.cjoint_forward(P, XV, XE)
    np.testing.assert_allclose(zj, _np_compact(P, np.concatenate([XV, np.zeros((40, 6))], 1), XE),
                               rtol=1e-12, atol=1e-12)


def _bf16_rne(x):
    """Round to BF16 (nearest, ties to even) through the FP32 bit pattern."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def test_compact_bf16_emulation(orc):
    """BF16 second layer of the compact MLP: equals a NumPy chain with
    bit-level rounding of the FP32 first-layer activations and of W2; with
    W2 already on the BF16 grid and activations made exact the two forms
    agree with the FP64 logits."""
    g = np.random.default_rng(21)
    P = synth.compact_params(g).astype(np.float64)
    X = g.uniform(-1, 1, (256, 16))
    o = 32 * 16 + 32
    W1, b1 = P[:512].reshape(32, 16), P[512:o]
    W2, b2 = P[o:o + 1024].reshape(32, 32), P[o + 1024:o + 1056]
    wo, bo = P[o + 1056:o + 1088], P[o + 1088]
    h = _bf16_rne(np.maximum(X @ W1.T + b1, 0).astype(np.float32))
    ref = np.maximum(h @ _bf16_rne(W2).T + b2, 0) @ wo + bo
    z = orc.cmlp_forward_bf16(P, X)
    np.testing.assert_allclose(z, ref, rtol=1e-12, atol=1e-12)
    z64, _ = orc.cmlp_forward(P, X)
    assert np.max(np.abs(z - z64)) > 1e-6  # the rounding is there
    # layer-1 weights zero but the bias, on the BF16 grid: no rounding left
    Q = P.copy()
    Q[:512] = 0.0
    Q[512:o] = _bf16_rne(np.abs(Q[512:o]))
    Q[o:o + 1024] = _bf16_rne(Q[o:o + 1024])
    np.testing.assert_allclose(orc.cmlp_forward_bf16(Q, X), orc.cmlp_forward(Q, X)[0], rtol=1e-12, atol=1e-12)


def test_compact_embedding_inputs_and_quaternion_sign(orc):
    q = (0.3, -0.5, 0.2, 0.7)
    a = one_gaussian_asset((0, 0, 0), (0.02, 0.03, 0.05), quat=q, opacity=0.6)
    b = one_gaussian_asset((0, 0, 0), (0.02, 0.03, 0.05), quat=tuple(-np.float32(v) for v in q), opacity=0.6)
    P = synth.compact_params(np.random.default_rng(1))
    for x in (a, b):
        x.mlp = synth.MLPSpec(params=P, width=32, bands=0, kind=1)
    Ea, XEa = orc.cembed(a)
    Eb, XEb = orc.cembed(b)
    qn = np.float32(q).astype(np.float64) / np.linalg.norm(np.float32(q).astype(np.float64))
    assert abs(XEa[0, 0] - np.float32(0.6)) < 1e-12
    np.testing.assert_allclose(XEa[0, 1:4], np.log(np.float32([0.02, 0.03, 0.05]).astype(np.float64)), atol=1e-12)
    np.testing.assert_allclose(XEa[0, 4:], qn, atol=1e-12)
    np.testing.assert_array_equal(XEa, XEb)  # q and -q: the same rotation, the same embedding
    np.testing.assert_array_equal(Ea, Eb)


def test_compact_inputs_closed_form_and_invariance(orc):
    """Identity instance, camera on the x axis at distance D looking at the
    origin: a Gaussian at the origin sees direction (-1, 0, 0), forward
    (-1, 0, 0) and distance D f_t / f_r mapped to [-1, 1]; an instance scaled
    by s at the same camera distance halves / scales that distance, and a
    rigid motion of camera and instance together changes no input."""
    D, res, fov = 6.0, 96, 50.0
    cam = synth.camera((D, 0.0, 0.0), width=res, height=res, fovy_deg=fov)
    a = one_gaussian_asset((0, 0, 0), (0.02, 0.03, 0.05))
    ft = float(np.float32(0.5 * 512 / math.tan(math.radians(fov) / 2)))
    a.mlp = synth.MLPSpec(params=synth.compact_params(np.random.default_rng(2)), width=32, bands=0,
                          mean_scale=0.5, train_focal=ft, d_min=2.0, d_max=50.0, kind=1)
    fr = 0.5 * res / math.tan(float(np.float32(math.radians(fov))) / 2)
    x = orc.cinputs(a, synth.identity_instance(0), cam, [0])[0]
    np.testing.assert_allclose(x[:3], 0.0, atol=1e-15)
    np.testing.assert_allclose(x[3:6], [-1, 0, 0], atol=1e-12)
    np.testing.assert_allclose(x[7:10], [-1, 0, 0], atol=1e-6)
    dt = D * ft / fr
    assert abs(x[6] - (2 * (dt - 2.0) / 48.0 - 1)) < 1e-9
    # an instance scaled by 2 at the origin: the local distance halves
    inst2 = Instance(asset=0, R=np.eye(3, dtype=np.float32), s=2.0, t=np.zeros(3, np.float32))
    x2 = orc.cinputs(a, inst2, cam, [0])[0]
    assert abs(x2[6] - (2 * (dt / 2 - 2.0) / 48.0 - 1)) < 1e-9
    # rigid motion of the world (exactly representable: a 90 degree yaw and an integer shift)
    Rz = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], np.float32)
    inst3 = Instance(asset=0, R=Rz, s=1.0, t=np.array([3, -2, 1], np.float32))
    cam3 = Camera(pos=(Rz.astype(np.float64) @ cam.pos.astype(np.float64) + [3, -2, 1]).astype(np.float32),
                  R=(cam.R.astype(np.float64) @ Rz.T.astype(np.float64)).astype(np.float32), fovy=cam.fovy,
                  width=res, height=res)
    x3 = orc.cinputs(a, inst3, cam3, [0])[0]
    np.testing.assert_allclose(x3, x, atol=1e-6)
    # far beyond the range the distance input saturates at 1
    far = synth.camera((500.0, 0.0, 0.0), width=res, height=res, fovy_deg=fov)
    assert orc.cinputs(a, synth.identity_instance(0), far, [0])[0][6] == 1.0


def test_compact_backward_central_differences(orc):
    g = np.random.default_rng(11)
    P = synth.compact_params(g).astype(np.float64)
    B = 24
    XV = np.concatenate([g.uniform(-1, 1, (B, 3)), g.standard_normal((B, 3)), g.uniform(-1, 1, (B, 1)),
                         g.standard_normal((B, 3))], 1)
    XE = np.concatenate([g.uniform(0.1, 1, (B, 1)), g.normal(-4.5, 0.3, (B, 3)), g.standard_normal((B, 4))], 1)
    y = (g.uniform(0, 1, B) > 0.5).astype(np.float64)
    w = g.uniform(0.5, 2.0, B)
    loss, dP = orc.cbce_backward(P, XV, XE, y, w)

    def pre_acts(Pp):
        # every hidden pre-activation of the batch (to skip parameters whose step crosses a ReLU kink)
        o = 0
        def take(r, c):
            nonlocal o
            W = Pp[o:o + r * c].reshape(r, c); o += r * c
            b = Pp[o:o + r]; o += r
            return W, b
        W1, b1 = take(32, 16); W2, b2 = take(32, 32); take(1, 32)
        E1, e1 = take(32, 8); E2, e2 = take(32, 32); E3, e3 = take(6, 32)
        a1 = XE @ E1.T + e1; a2 = np.maximum(a1, 0) @ E2.T + e2
        emb = np.maximum(a2, 0) @ E3.T + e3
        X = np.concatenate([XV, emb], 1)
        v1 = X @ W1.T + b1; v2 = np.maximum(v1, 0) @ W2.T + b2
        return np.concatenate([a1.ravel(), a2.ravel(), v1.ravel(), v2.ravel()])

    eps = 1e-3
    base = np.sign(pre_acts(P))
    checked = 0
    for k in range(P.size):
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += eps; Pm[k] -= eps
        if not (np.array_equal(np.sign(pre_acts(Pp)), base) and np.array_equal(np.sign(pre_acts(Pm)), base)):
            continue
        lp, _ = orc.cbce_backward(Pp, XV, XE, y, w)
        lm, _ = orc.cbce_backward(Pm, XV, XE, y, w)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - dP[k]) <= 1e-3 * max(abs(dP[k]), 1e-6 * np.abs(dP).max()) + 1e-9, k
        checked += 1
    assert checked > 0.9 * P.size
    # the loss itself
    z = _np_compact(P, XV, XE)
    assert abs(loss - np.mean(w * (np.logaddexp(0, z) - z * y))) < 1e-12


def test_compact_query_gate(orc):
    """Below the minimum distance every in-frustum Gaussian is kept without a
    query; beyond it the keep decision is the sign of the compact MLP's logit."""
    a = synth.make_asset("sphere", 400, 0, 77, width=16)
    # 48 px views with the 512 px training focal: distances are corrected by about 11.4
    a = synth.make_compact(a, seed=5, d_min=40.0, d_max=200.0)
    near = synth.camera((0.0, -2.5, 0.5), width=48, height=48)   # corrected ~29 < d_min
    far = synth.camera((0.0, -6.0, 1.0), width=48, height=48)    # corrected ~69 > d_min
    sc = Scene(assets=[a], instances=[synth.identity_instance(0)], cameras=[near, far])
    st, lg = orc.query(sc)
    inside = st > 0
    assert inside[0].any() and inside[1].any()
    assert np.all(st[0][inside[0]] == 2) and np.all(np.isnan(lg[0]))
    q = inside[1]
    X = orc.cinputs(a, synth.identity_instance(0), far, np.flatnonzero(q))
    z, _ = orc.cmlp_forward(a.mlp.params, X)
    np.testing.assert_array_equal(lg[1][q], z)
    np.testing.assert_array_equal(st[1][q] == 2, z >= 0)


def test_per_splat_decision_margins(orc):
    """Per-splat margins of the decisions that decide a splat's contribution:
    the three-opaque-splats case, where the second blend lands T exactly on
    1e-4 (a knife edge), so every splat tested at or listed after that
    decision carries its near-zero margin; the first splat's only decisions
    are far from their thresholds (alpha 0.99, then T = 0.01: relative
    margin 99 to 1e-4).  The splats are wide, so every pixel holds the stack."""
    cam = axis_camera(4, 4)
    rec = np.stack([_rec(1.5, 1.5, 1e6, 0, 1e6, 1.0 + k, 1.0, (1.0, 1.0, 1.0)) for k in range(4)])
    sm = np.full((4, 2), np.inf)
    orc.render_camera(rec, _full_rect(4, 4, 4), cam, 4, smargin=sm)
    assert abs(sm[0, 0] - 99.0) < 1e-9 and sm[0, 1] == np.inf
    assert np.all(sm[1:, 0] < 1e-10)
    # depth gaps: (2 - 1) / 2 at the second splat, then (3 - 2) / 3, and at
    # the stop the gap to the next fragment, (4 - 3) / 4
    assert abs(sm[1, 1] - 0.5) < 1e-15 and abs(sm[2, 1] - 0.25) < 1e-15 and abs(sm[3, 1] - 0.25) < 1e-15
    # the same stack without the knife edge (first alpha 0.9): wide margins,
    # and the never-reached fourth splat inherits the stop decision's margin
    rec[0, 9] = 0.9
    sm = np.full((4, 2), np.inf)
    rc = np.zeros(4, np.uint8)
    orc.render_camera(rec, _full_rect(4, 4, 4), cam, 4, reached=rc, smargin=sm)
    # T: 1 -> 0.1 -> 0.001 -> 1e-5 < 1e-4 (third splat stops the pixel)
    assert rc.tolist() == [1, 1, 1, 0]
    # (the off-centre pixels see alpha lower by ~1e-6 relative: the splat is
    # wide, not infinite)
    stop_margin = abs(0.1 * 0.01 * 0.01 - 1e-4) / 1e-4
    assert abs(sm[3, 0] - min(stop_margin, abs(0.001 - 1e-4) / 1e-4, abs(0.1 - 1e-4) / 1e-4)) < 1e-4
    assert abs(sm[0, 0] - (0.9 - 1 / 255) * 255) < 1e-2


def test_depth_margin_covers_the_fragment_after_the_stop(orc):
    """The pixel stops at the third splat; a fourth lies 1e-7 (relative)
    behind it.  A renderer whose depth keys tie the two may blend the fourth
    before the stop, so the pixel's depth margin (and the fourth splat's) is
    that gap, not the 1/3 between the blended ones."""
    cam = axis_camera(4, 4)
    specs = [(1.0, 1.0), (2.0, 0.9), (3.0, 0.95), (3.0 * (1 + 1e-7), 0.5)]  # depth, opacity
    rec = np.stack([_rec(1.5, 1.5, 1e6, 0, 1e6, dep, o, (1.0, 1.0, 1.0)) for dep, o in specs])
    sm = np.full((4, 2), np.inf)
    rc = np.zeros(4, np.uint8)
    out = orc.render_camera(rec, _full_rect(4, 4, 4), cam, 4, reached=rc, smargin=sm)
    # T: 1 -> 0.01 -> 0.001 -> 5e-5 < 1e-4: the third splat stops the pixel
    assert rc.tolist() == [1, 1, 1, 0]
    gap = 3.0 * 1e-7 / (3.0 * (1 + 1e-7))
    assert abs(out["margin"][1, 1, 1] - gap) < 1e-15
    assert abs(sm[3, 1] - gap) < 1e-15 and abs(sm[2, 1] - gap) < 1e-15 and abs(sm[1, 1] - 0.5) < 1e-15
