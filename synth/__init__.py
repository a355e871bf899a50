"""Seeded synthetic inputs for the NVGS per-frame path.

This module only *draws* inputs: Gaussian assets, instance transforms,
cameras and MLP weights.  It holds none of the method's arithmetic (no
culling, encoding, MLP evaluation, projection or blending); both the HIP
path and the CPU oracle consume its arrays unchanged.

Layout of one asset (all float32, structure-of-arrays):

* ``mean``    [3, N]   Gaussian centres in the asset frame
* ``scale``   [3, N]   linear per-axis standard deviations
* ``quat``    [4, N]   unit quaternion (w, x, y, z)
* ``opacity`` [N]      activated opacity in (0, 1]
* ``sh``      [K*3, N] spherical-harmonic coefficients, plane ``c*3 + ch``
  for coefficient ``c`` (l-major, m = -l..l) and colour channel ``ch``;
  K = (degree + 1)^2

The visibility MLP is a packed float32 vector: W1 [W, 72], b1 [W],
W2 [W, W], b2 [W], W3 [W, W], b3 [W], wo [W], bo [1] (row-major).

Scene recipes follow the workloads the paper measures (composed scenes of
separately trained assets, Sec. 4.2 and the supplementary per-asset and
large-scene sections); the paper's own datasets are not available, so these
generated shapes stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

# Real SH basis, l = 0: Y00 = 1 / (2 sqrt(pi)).  Used only to store an RGB
# colour as a degree-0 coefficient (input preparation, not rendering).
_Y00 = 0.5 / math.sqrt(math.pi)

SEED_BASE = 20251119


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# data containers
# ----------------------------------------------------------------------------
@dataclass
class MLPSpec:
    params: np.ndarray          # float32 packed blob
    width: int = 64
    bands: int = 6
    mean_scale: float = 0.5     # sigma_mu
    cam_scale: float = 0.05     # sigma_c
    train_focal: float = 548.9  # focal length (pixels) of the training views: (H/2) / tan(fovy/2)
    d_min: float = 0.0          # minimum-distance gate (0 = off)
    d_max: float = 0.0          # far clamp of the local camera distance (0 = off)
    kind: int = 0               # 0: frequency-encoded 72-input MLP; 1: the compact 16-input form


@dataclass
class Asset:
    mean: np.ndarray
    scale: np.ndarray
    quat: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    sh_degree: int
    mlp: MLPSpec
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])


@dataclass
class Instance:
    asset: int
    R: np.ndarray               # float32 [3, 3] asset -> world rotation
    s: float                    # uniform scale
    t: np.ndarray               # float32 [3] translation


@dataclass
class Camera:
    pos: np.ndarray             # float32 [3]
    R: np.ndarray               # float32 [3, 3] world -> camera, rows right, down, forward
    fovy: float                 # radians, vertical
    width: int
    height: int
    near: float = 0.2


@dataclass
class Scene:
    assets: List[Asset]
    instances: List[Instance]
    cameras: List[Camera]
    tile: int = 16
    bg: tuple = (0.0, 0.0, 0.0)
    name: str = ""
    extra: dict = field(default_factory=dict)

    def pair_offsets(self) -> np.ndarray:
        """Start of each instance's Gaussians in the per-camera pair index."""
        sizes = [self.assets[i.asset].n for i in self.instances]
        return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)

    @property
    def pairs_per_camera(self) -> int:
        return int(self.pair_offsets()[-1])


# ----------------------------------------------------------------------------
# parameter draws
# ----------------------------------------------------------------------------
def mlp_params(width: int, g: np.random.Generator, in_dim: int = 72, hidden: int = 3) -> np.ndarray:
    """U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for every weight and bias."""
    parts = []
    fan = in_dim
    for _ in range(hidden):
        b = 1.0 / math.sqrt(fan)
        parts.append(g.uniform(-b, b, size=(width, fan)).ravel())
        parts.append(g.uniform(-b, b, size=width))
        fan = width
    b = 1.0 / math.sqrt(fan)
    parts.append(g.uniform(-b, b, size=width))
    parts.append(g.uniform(-b, b, size=1))
    return np.concatenate(parts).astype(np.float32)


COMPACT_VIS_PARAMS = 32 * 16 + 32 + 32 * 32 + 32 + 32 + 1
COMPACT_EMB_PARAMS = 32 * 8 + 32 + 32 * 32 + 32 + 6 * 32 + 6


def compact_params(g: np.random.Generator) -> np.ndarray:
    """The compact form's packed parameters (visibility 16-32-32-1, then the
    embedding 8-32-32-6), each layer U(-1/sqrt(fan_in), 1/sqrt(fan_in))."""
    parts = []
    for rows, fan in ((32, 16), (32, 32), (1, 32), (32, 8), (32, 32), (6, 32)):
        b = 1.0 / math.sqrt(fan)
        parts.append(g.uniform(-b, b, size=(rows, fan)).ravel())
        parts.append(g.uniform(-b, b, size=rows))
    return np.concatenate(parts).astype(np.float32)


def make_compact(asset, seed: int, d_min: float, d_max: float):
    """The asset with the compact MLP form (seeded weights), normalising the
    camera distance over [d_min, d_max]."""
    import copy
    a = copy.copy(asset)
    a.mlp = MLPSpec(params=compact_params(rng(seed)), width=32, bands=0, mean_scale=asset.mlp.mean_scale,
                    cam_scale=0.0, train_focal=asset.mlp.train_focal, d_min=d_min, d_max=d_max, kind=1)
    return a


def mlp_param_count(width: int, in_dim: int = 72, hidden: int = 3) -> int:
    n = in_dim * width + width
    n += (hidden - 1) * (width * width + width)
    return n + width + 1


def random_quats(n: int, g: np.random.Generator) -> np.ndarray:
    q = g.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q.astype(np.float32)


def gaussian_params(means: np.ndarray, g: np.random.Generator, sh_degree: int,
                    scale_mu: float = -4.5, scale_sigma: float = 0.3,
                    opacity_lo: float = 0.3, sh_std: float = 0.1):
    n = means.shape[1]
    scale = np.exp(g.normal(scale_mu, scale_sigma, size=(3, n))).astype(np.float32)
    quat = random_quats(n, g)
    opacity = g.uniform(opacity_lo, 1.0, size=n).astype(np.float32)
    k = (sh_degree + 1) ** 2
    if sh_degree == 0:
        rgb = g.uniform(0.0, 1.0, size=(3, n))
        sh = ((rgb - 0.5) / _Y00).astype(np.float32)
    else:
        sh = g.normal(0.0, sh_std, size=(k * 3, n)).astype(np.float32)
    return scale, quat, opacity, sh


# ----------------------------------------------------------------------------
# shapes (means only)
# ----------------------------------------------------------------------------
def torus_means(n, g, R=1.0, r=0.35, jitter=0.01, normals=False):
    """Area-uniform torus surface (axis +z) plus N(0, jitter^2) jitter (and the
    unit surface normals [3, n] of the points before jitter if `normals`)."""
    out_u = np.empty(0)
    out_v = np.empty(0)
    while out_u.size < n:
        m = 2 * (n - out_u.size) + 64
        u = g.uniform(0, 2 * np.pi, m)
        v = g.uniform(0, 2 * np.pi, m)
        w = g.uniform(0, 1, m)
        ok = w <= (R + r * np.cos(v)) / (R + r)
        out_u = np.concatenate([out_u, u[ok]])
        out_v = np.concatenate([out_v, v[ok]])
    u, v = out_u[:n], out_v[:n]
    x = (R + r * np.cos(v)) * np.cos(u)
    y = (R + r * np.cos(v)) * np.sin(u)
    z = r * np.sin(v)
    p = np.stack([x, y, z]) + g.normal(0, jitter, size=(3, n))
    if normals:
        return p.astype(np.float32), np.stack([np.cos(v) * np.cos(u), np.cos(v) * np.sin(u), np.sin(v)])
    return p.astype(np.float32)


def sphere_means(n, g, radius=1.0, jitter=0.01, normals=False):
    d = g.standard_normal((3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    p = (radius * d + g.normal(0, jitter, size=(3, n))).astype(np.float32)
    return (p, d) if normals else p


def box_means(n, g, half=1.0, jitter=0.01, normals=False):
    face = g.integers(0, 6, n)
    a = g.uniform(-half, half, n)
    b = g.uniform(-half, half, n)
    p = np.zeros((3, n))
    axis = face // 2
    sign = np.where(face % 2 == 0, -1.0, 1.0)
    for ax in range(3):
        sel = axis == ax
        o1, o2 = [k for k in range(3) if k != ax]
        p[ax, sel] = sign[sel] * half
        p[o1, sel] = a[sel]
        p[o2, sel] = b[sel]
    q = (p + g.normal(0, jitter, size=(3, n))).astype(np.float32)
    if normals:
        nrm = np.zeros((3, n))
        nrm[axis, np.arange(n)] = sign
        return q, nrm
    return q


def helix_means(n, g, radius=0.8, pitch=0.15, turns=3.0, tube=0.15, jitter=0.01, normals=False):
    th = g.uniform(0, 2 * np.pi * turns, n)
    ph = g.uniform(0, 2 * np.pi, n)
    c = np.stack([radius * np.cos(th), radius * np.sin(th), pitch * th - pitch * np.pi * turns])
    t = np.stack([-radius * np.sin(th), radius * np.cos(th), np.full(n, pitch)])
    t /= np.linalg.norm(t, axis=0, keepdims=True)
    nrm = np.stack([-np.cos(th), -np.sin(th), np.zeros(n)])
    bin_ = np.cross(t.T, nrm.T).T
    out = np.cos(ph) * nrm + np.sin(ph) * bin_
    p = c + tube * out
    q = (p + g.normal(0, jitter, size=(3, n))).astype(np.float32)
    return (q, out / np.linalg.norm(out, axis=0, keepdims=True)) if normals else q


SHAPES = {"torus": torus_means, "sphere": sphere_means, "box": box_means, "helix": helix_means}
# half bounding-box diagonals of the four shapes (jitter ignored)
SHAPE_HALF_DIAG = {
    "torus": math.sqrt(1.35 ** 2 * 2 + 0.35 ** 2),
    "sphere": math.sqrt(3.0),
    "box": math.sqrt(3.0),
    "helix": math.sqrt(0.95 ** 2 * 2 + (0.15 * math.pi * 3 + 0.15) ** 2),
}


def pow2_scale(r: float) -> float:
    """Largest power of two s with s * r <= 1 (exact scaling in binary FP)."""
    return 2.0 ** (-math.ceil(math.log2(r)))


def surface_frames(normals: np.ndarray, g: np.random.Generator) -> np.ndarray:
    """Unit quaternions (w, x, y, z), [4, n], of rotations whose third axis is
    the given normal, with a uniform random twist about it: the shortest-arc
    rotation from +z to the normal composed with a rotation about +z."""
    nz = normals / np.linalg.norm(normals, axis=0, keepdims=True)
    n = nz.shape[1]
    # shortest arc z -> n: (1 + z.n, z x n) normalised; the antipode takes a half turn about x
    q1 = np.stack([1.0 + nz[2], -nz[1], nz[0], np.zeros(n)])
    flip = nz[2] < -1.0 + 1e-9
    q1[:, flip] = np.array([[0.0], [1.0], [0.0], [0.0]])
    q1 /= np.linalg.norm(q1, axis=0, keepdims=True)
    psi = g.uniform(0, 2 * np.pi, n)
    c, s_ = np.cos(psi / 2), np.sin(psi / 2)
    w1, x1, y1, z1 = q1
    # q1 * (c, 0, 0, s)
    q = np.stack([w1 * c - z1 * s_, x1 * c + y1 * s_, y1 * c - x1 * s_, z1 * c + w1 * s_])
    return q.astype(np.float32)


def make_asset(shape: str, n: int, sh_degree: int, seed: int, width: int = 64,
               cam_scale: float = 0.05, fov_train: float = math.radians(50.0), res_train: int = 512,
               d_max: float = 20.0, aligned: bool = False) -> Asset:
    """One synthetic asset.  aligned: the Gaussians are flat discs lying in
    the surface (as in optimised 3DGS assets): the scale along the surface
    normal shrunk 10x and the rotation's third axis on the normal (random
    twist); otherwise random orientations with independent per-axis scales."""
    g = rng(seed)
    means, normals = SHAPES[shape](n, g, normals=True)
    scale, quat, opacity, sh = gaussian_params(means, g, sh_degree)
    if aligned:
        g2 = rng(seed + 7919)
        scale = scale.copy()
        scale[2] *= np.float32(0.1)
        quat = surface_frames(normals, g2)
    params = mlp_params(width, g)
    spec = MLPSpec(params=params, width=width, bands=6,
                   mean_scale=pow2_scale(SHAPE_HALF_DIAG[shape]), cam_scale=cam_scale,
                   train_focal=float(np.float32(0.5 * res_train / math.tan(float(np.float32(fov_train)) / 2.0))),
                   d_min=0.0, d_max=d_max)
    return Asset(mean=means, scale=scale, quat=quat, opacity=opacity, sh=sh,
                 sh_degree=sh_degree, mlp=spec, name=shape)


# ----------------------------------------------------------------------------
# cameras and instances
# ----------------------------------------------------------------------------
def look_at(pos, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World->camera rotation with rows (right, down, forward)."""
    pos = np.asarray(pos, np.float64)
    f = np.asarray(target, np.float64) - pos
    f /= np.linalg.norm(f)
    up = np.asarray(up, np.float64)
    if abs(np.dot(f, up)) > 0.999:
        up = np.array([0.0, 1.0, 0.0])
    right = np.cross(f, up)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    return np.stack([right, down, f]).astype(np.float32)


def camera(pos, target=(0, 0, 0), fovy_deg=50.0, width=256, height=256, near=0.2) -> Camera:
    return Camera(pos=np.asarray(pos, np.float32), R=look_at(pos, target),
                  fovy=math.radians(fovy_deg), width=width, height=height, near=near)


def yaw(theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], np.float32)


def identity_instance(asset: int = 0) -> Instance:
    return Instance(asset=asset, R=np.eye(3, dtype=np.float32), s=1.0, t=np.zeros(3, np.float32))


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def scene_tiny(n: int = 20000, seed: int = SEED_BASE + 1, width: int = 64,
               res: int = 256, tile: int = 16) -> Scene:
    """1 torus asset (SH0), 1 identity instance, 1 camera at distance 3, 30 deg elevation."""
    a = make_asset("torus", n, 0, seed * 100 + 0, width=width)
    el = math.radians(30.0)
    cam = camera((0.0, -3.0 * math.cos(el), 3.0 * math.sin(el)), fovy_deg=50.0, width=res, height=res)
    return Scene(assets=[a], instances=[identity_instance(0)], cameras=[cam], tile=tile, name="tiny")


def scene_composed(n_per_asset: int = 250000, n_inst: int = 64, seed: int = SEED_BASE + 2,
                   width: int = 64, res=(1920, 1080), tile: int = 16, sh_degree: int = 3,
                   half_extent: float = 20.0, aligned: bool = False) -> Scene:
    """4 assets (torus, sphere shell, box shell, helix tube), SH3; n_inst
    instances with random yaw, scale U(0.5, 2), positions U(-20, 20)^2 at z=0;
    one camera at (0, -30, 12) looking at the origin.  aligned: surface-aligned
    flat Gaussians (see make_asset)."""
    names = ["torus", "sphere", "box", "helix"]
    assets = [make_asset(nm, n_per_asset, sh_degree, seed * 100 + j, width=width, aligned=aligned)
              for j, nm in enumerate(names)]
    g = rng(seed)
    insts = []
    for i in range(n_inst):
        th = g.uniform(0, 2 * np.pi)
        s = g.uniform(0.5, 2.0)
        xy = g.uniform(-half_extent, half_extent, 2)
        insts.append(Instance(asset=i % 4, R=yaw(th), s=float(np.float32(s)),
                              t=np.array([xy[0], xy[1], 0.0], np.float32)))
    cam = camera((0.0, -30.0, 12.0), fovy_deg=50.0, width=res[0], height=res[1])
    return Scene(assets=assets, instances=insts, cameras=[cam], tile=tile, name="composed")


def scene_batched(n_assets: int = 16, n_inst: int = 1024, n_cams: int = 8,
                  seed: int = SEED_BASE + 4, width: int = 64, res=(1920, 1080),
                  tile: int = 16, sh_degree: int = 3, n_lo: float = 5e4, n_hi: float = 1e6,
                  half_extent: float = 80.0, frame: int = 0, size_scale: float = 1.0,
                  ring_radius: float = 60.0, ring_height: float = 15.0) -> Scene:
    """Uneven assets (log-uniform sizes), Zipf instance counts, a ring of
    cameras looking at the centre, turned by `frame` degrees."""
    names = ["torus", "sphere", "box", "helix"]
    g = rng(seed)
    sizes = np.round(np.exp(g.uniform(math.log(n_lo), math.log(n_hi), n_assets)) * size_scale).astype(np.int64)
    sizes = np.maximum(sizes, 1)
    w = 1.0 / np.arange(1, n_assets + 1)
    counts = np.floor(w / w.sum() * n_inst).astype(np.int64)
    counts[0] += n_inst - counts.sum()
    perm = g.permutation(n_assets)
    per_asset = np.zeros(n_assets, np.int64)
    per_asset[perm] = counts
    assets = [make_asset(names[j % 4], int(sizes[j]), sh_degree, seed * 100 + j, width=width)
              for j in range(n_assets)]
    insts = []
    for a in range(n_assets):
        for _ in range(int(per_asset[a])):
            th = g.uniform(0, 2 * np.pi)
            s = g.uniform(0.5, 2.0)
            xy = g.uniform(-half_extent, half_extent, 2)
            insts.append(Instance(asset=a, R=yaw(th), s=float(np.float32(s)),
                                  t=np.array([xy[0], xy[1], 0.0], np.float32)))
    order = g.permutation(len(insts))
    insts = [insts[k] for k in order]
    cams = ring_cameras(n_cams, frame, ring_radius, ring_height, res)
    return Scene(assets=assets, instances=insts, cameras=cams, tile=tile, name="batched",
                 extra={"instances_per_asset": per_asset.tolist(), "sizes": sizes.tolist()})


def ring_cameras(n_cams: int = 8, frame: float = 0.0, radius: float = 60.0, height: float = 15.0,
                 res=(1920, 1080), fovy_deg: float = 50.0) -> List[Camera]:
    """n_cams cameras evenly spaced on a horizontal circle, looking at the
    origin, the ring turned by `frame` degrees."""
    cams = []
    for k in range(n_cams):
        ang = 2 * np.pi * k / n_cams + math.radians(frame)
        cams.append(camera((radius * math.cos(ang), radius * math.sin(ang), height), fovy_deg=fovy_deg,
                           width=res[0], height=res[1]))
    return cams


def eq1_range(shape: str, fovy_deg: float = 50.0, near: float = 0.9, far: float = 0.05):
    """Eq. 1 camera-distance range of an asset: the distance at which its
    bounding-box diagonal covers `near` and `far` of the image, d = r /
    (tan(fov/2) p), r the half-diagonal."""
    t = math.tan(math.radians(fovy_deg) / 2)
    r = SHAPE_HALF_DIAG[shape]
    return r / (t * near), r / (t * far)


def fibonacci_sphere(n: int) -> np.ndarray:
    """n unit directions on the Fibonacci (golden-angle) spiral, [n, 3]."""
    k = np.arange(n, dtype=np.float64) + 0.5
    z = 1.0 - 2.0 * k / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def longlat_sphere(n: int) -> np.ndarray:
    """About n unit directions on a longitude-latitude grid (equal angular
    steps, so denser towards the poles), [n, 3]: ceil(sqrt(n / 2)) latitude
    rings at cell centres, 2x as many longitudes, truncated to n."""
    n_lat = max(1, math.ceil(math.sqrt(n / 2)))
    n_lon = max(1, math.ceil(n / n_lat))
    lat = -math.pi / 2 + math.pi * (np.arange(n_lat) + 0.5) / n_lat
    lon = 2 * math.pi * np.arange(n_lon) / n_lon
    la, lo = np.meshgrid(lat, lon, indexing="ij")
    d = np.stack([np.cos(la) * np.cos(lo), np.cos(la) * np.sin(lo), np.sin(la)], axis=-1).reshape(-1, 3)
    return d[:n]


def label_views(n_views: int, seed: int, d_lo: float = 1.5, d_hi: float = 20.0,
                res: int = 512, fovy_deg: float = 50.0, offset: float = 0.0, sampling: str = "fibonacci",
                radius: float = 1.0) -> List[Camera]:
    """Training views (Sec. 3.1, 4.1 recipe): Fibonacci-sphere directions (or
    a longitude-latitude grid, the ablation's baseline), distance U(d_lo,
    d_hi) per view, looking at the asset centre displaced by a random offset:
    none at d_lo, growing linearly with the distance to at most
    `offset` * radius * d_hi / d_lo at d_hi, uniform in that ball.  With
    offset 1 and the asset's half-diagonal as radius, an asset at d_hi (where
    it covers p_far of the image) moves by up to (p_near / p_far) radii, so it
    stays in the frame at every distance."""
    g = rng(seed)
    d = fibonacci_sphere(n_views) if sampling == "fibonacci" else longlat_sphere(n_views)
    r = g.uniform(d_lo, d_hi, n_views)
    u = g.standard_normal((n_views, 3))
    u *= (g.uniform(0.0, 1.0, n_views) ** (1.0 / 3.0) / np.linalg.norm(u, axis=1))[:, None]
    lam = (r - d_lo) / max(d_hi - d_lo, 1e-12)
    off = u * (offset * radius * (d_hi / d_lo) * lam)[:, None]
    return [camera(d[k] * r[k], target=tuple(off[k]), fovy_deg=fovy_deg, width=res, height=res)
            for k in range(n_views)]


def scene_train(n: int = 500000, seed: int = SEED_BASE + 5, width: int = 64, sh_degree: int = 3) -> Scene:
    a = make_asset("torus", n, sh_degree, seed * 100 + 0, width=width, cam_scale=1.0 / 20.0, d_max=20.0,
                   res_train=512)
    return Scene(assets=[a], instances=[identity_instance(0)], cameras=[], tile=16, name="train")
