"""FP64 CPU oracle for the NVGS per-frame path (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It never imports the product package
and the product never imports it; the two share only the seeded inputs of
``synth``.

The heavy loops live in ``nvgs_oracle.cpp`` (plain C++17, FP64, no FMA
contraction, OpenMP over independent outputs).  This file marshals the
``synth`` containers into flat arrays and strings the steps together in the
order of the method (Sec. 3.3): frustum cull -> MLP query -> compaction of the
survivors -> projection -> (tile, depth, id) ordering -> compositing.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nvgs_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

REC = 16  # doubles per projected splat record (see nvgs_oracle.cpp)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off",
                               "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        fp = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        u8 = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        i32 = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64 = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        vp = C.c_void_p
        L.orc_encode.argtypes = [dp, C.c_int, C.c_int, dp]
        L.orc_encode_batch.argtypes = [dp, C.c_int64, C.c_int, C.c_int, dp]
        L.orc_mlp_forward.argtypes = [dp, C.c_int, C.c_int, dp, C.c_int64, dp, vp, vp]
        L.orc_sh_basis.argtypes = [dp, C.c_int, dp]
        L.orc_local_camera.argtypes = [dp, dp, C.c_double, C.c_double, dp]
        L.orc_query.argtypes = [C.c_int64, fp, dp, dp, dp, C.c_int, C.c_int, C.c_double, C.c_double,
                                C.c_double, C.c_double, C.c_double, C.c_int, u8, dp, vp]
        L.orc_project.argtypes = [C.c_int64, i64, C.c_int64, fp, fp, fp, fp, fp, C.c_int, dp, dp, dp, i32]
        L.orc_render.argtypes = [C.c_int64, dp, i32, dp, C.c_int, dp, dp, vp, vp, vp, vp, vp, C.c_int64, vp]
        L.orc_render.restype = C.c_int64
        L.orc_render_brute.argtypes = [C.c_int64, dp, dp, dp, dp, vp]
        L.orc_bce_backward.argtypes = [dp, C.c_int, C.c_int, dp, dp, vp, C.c_int64, dp, vp]
        L.orc_bce_backward.restype = C.c_double
        L.orc_adam_step.argtypes = [C.c_int64, dp, dp, dp, dp, C.c_int64, C.c_double, C.c_double,
                                    C.c_double, C.c_double]
        L.orc_fp8_scales.argtypes = [dp, C.c_int, dp]
        L.orc_mlp_forward_q.argtypes = [dp, C.c_int, dp, C.c_int64, C.c_int, dp]
        L.orc_to_bf16.argtypes = [C.c_double]
        L.orc_to_bf16.restype = C.c_double
        L.orc_to_e4m3.argtypes = [C.c_double]
        L.orc_to_e4m3.restype = C.c_double
        L.orc_lr_schedule.argtypes = [C.c_double, C.c_double, C.c_int64, C.c_int64]
        L.orc_lr_schedule.restype = C.c_double
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = C.c_int
        L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_compact_sizes.argtypes = [C.c_int]
        L.orc_compact_sizes.restype = C.c_int
        L.orc_cembed.argtypes = [C.c_int64, fp, fp, fp, dp, dp, vp]
        L.orc_cinputs.argtypes = [C.c_int64, i64, C.c_int64, fp, dp, dp, dp, C.c_double, C.c_double, C.c_double,
                                  C.c_double, dp]
        L.orc_cmlp_forward.argtypes = [dp, dp, C.c_int64, dp, vp]
        L.orc_cmlp_forward_bf16.argtypes = [dp, dp, C.c_int64, dp]
        L.orc_cjoint_forward.argtypes = [dp, dp, dp, C.c_int64, dp, vp]
        L.orc_cquery.argtypes = [C.c_int64, fp, dp, dp, dp, dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                 C.c_int, u8, dp, vp]
        L.orc_cbce_backward.argtypes = [dp, dp, dp, dp, vp, C.c_int64, dp]
        L.orc_cbce_backward.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
# records
# ----------------------------------------------------------------------------
def inst_array(inst) -> np.ndarray:
    """Instance record; every field passes through float32, the precision in
    which instances are handed over, then is widened exactly to FP64."""
    return _f64(np.concatenate([np.asarray(inst.R, np.float32).ravel(), np.float32([inst.s]),
                                np.asarray(inst.t, np.float32).ravel()]).astype(np.float32))


def cam_array(cam) -> np.ndarray:
    """Camera record (float32 fields widened exactly to FP64)."""
    return _f64(np.concatenate([np.asarray(cam.pos, np.float32).ravel(),
                                np.asarray(cam.R, np.float32).ravel(),
                                np.float32([cam.fovy, cam.width, cam.height, cam.near])]).astype(np.float32))


# ----------------------------------------------------------------------------
# single steps
# ----------------------------------------------------------------------------
def encode(x: np.ndarray, bands: int = 6) -> np.ndarray:
    x = _f64(x).ravel()
    out = np.zeros(x.size * bands * 2)
    lib().orc_encode(x, x.size, bands, out)
    return out


def mlp_forward(params, width: int, X: np.ndarray, want_pre: bool = False):
    """Logits of the packed MLP for inputs X [B, in_dim] (FP64)."""
    X = _f64(X)
    B, in_dim = X.shape
    z = np.zeros(B)
    sc = np.zeros(B)
    pre = np.zeros((B, 3 * width)) if want_pre else None
    lib().orc_mlp_forward(_f64(params), width, in_dim, X, B, z, _ptr(pre), _ptr(sc))
    return (z, sc, pre) if want_pre else (z, sc)


PREC = {"bf16": 1, "fp8": 2}


def mlp_forward_q(params, width: int, X: np.ndarray, prec: str) -> np.ndarray:
    """Logits of the MLP with its GEMM operands rounded to BF16 or FP8 E4M3."""
    X = _f64(X)
    z = np.zeros(X.shape[0])
    lib().orc_mlp_forward_q(_f64(params), width, X, X.shape[0], PREC[prec], z)
    return z


def fp8_scales(params, width: int) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_fp8_scales(_f64(params), width, out)
    return out


def to_bf16(x) -> np.ndarray:
    """BF16 round-to-nearest-even of float32(x), elementwise."""
    f = np.vectorize(lambda v: lib().orc_to_bf16(float(v)), otypes=[np.float64])
    return f(np.asarray(x, np.float64))


def to_e4m3(x) -> np.ndarray:
    """OCP E4M3 round-to-nearest-even with saturation at 448, elementwise."""
    f = np.vectorize(lambda v: lib().orc_to_e4m3(float(v)), otypes=[np.float64])
    return f(np.asarray(x, np.float64))


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops (n <= 0: all processors); returns the count now in use."""
    lib().orc_set_threads(int(n))
    return int(lib().orc_max_threads())


def lr_schedule(lr: float, lr_final: float, T: int, t: int) -> float:
    """Learning rate of step t of T under the warm-up + exponential decay schedule (Sec. 4.1)."""
    return float(lib().orc_lr_schedule(lr, lr_final, T, t))


def sh_basis(d, degree: int = 3) -> np.ndarray:
    Y = np.zeros(16)
    lib().orc_sh_basis(_f64(d), degree, Y)
    return Y[: (degree + 1) ** 2]


def local_camera(inst, cam, train_focal: float, d_max: float = 0.0) -> np.ndarray:
    out = np.zeros(3)
    lib().orc_local_camera(inst_array(inst), cam_array(cam), train_focal, d_max, out)
    return out


def mlp_inputs(asset, gidx: np.ndarray, cam_local: np.ndarray) -> np.ndarray:
    """Encoded MLP inputs (FP64) for Gaussians gidx seen from cam_local [.., 3]."""
    spec = asset.mlp
    mu = asset.mean[:, gidx].T.astype(np.float64) * spec.mean_scale
    cl = np.broadcast_to(np.asarray(cam_local, np.float64) * spec.cam_scale, mu.shape)
    x = np.ascontiguousarray(np.concatenate([mu, cl], axis=1))
    out = np.zeros((len(x), 12 * spec.bands))
    if len(x):
        lib().orc_encode_batch(x, len(x), 6, spec.bands, out)
    return out


def bce_backward(params, width: int, X, y, w=None, want_dx: bool = False):
    P = _f64(params)
    X = _f64(X)
    B, in_dim = X.shape
    dP = np.zeros_like(P)
    dX = np.zeros_like(X) if want_dx else None
    loss = lib().orc_bce_backward(P, width, in_dim, X, _f64(y), _ptr(None if w is None else _f64(w)),
                                  B, dP, _ptr(dX))
    return (loss, dP, dX) if want_dx else (loss, dP)


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays p, m, v with gradient g."""
    lib().orc_adam_step(p.size, p, _f64(g), m, v, t, lr, b1, b2, eps)


def splitmix64(seed: int, i: int) -> int:
    return int(lib().orc_splitmix64(seed, i))


# ----------------------------------------------------------------------------
# the per-frame path
# ----------------------------------------------------------------------------
def query(scene, use_mlp: bool = True, cams=None, want_margin: bool = False):
    """Cull + MLP query for every (camera, instance, Gaussian).

    Returns state [C, P] (0 frustum-culled, 1 MLP-culled, 2 kept),
    logits [C, P] (NaN where not queried) and optionally margins [C, P]."""
    cams = scene.cameras if cams is None else cams
    off = scene.pair_offsets()
    P = int(off[-1])
    state = np.zeros((len(cams), P), np.uint8)
    logit = np.full((len(cams), P), np.nan)
    margin = np.zeros((len(cams), P)) if want_margin else None
    params64 = [_f64(a.mlp.params) for a in scene.assets]
    embeds = [cembed(a)[0] if a.mlp.kind == 1 else None for a in scene.assets]
    L = lib()
    for k, cam in enumerate(cams):
        ca = cam_array(cam)
        for i, inst in enumerate(scene.instances):
            a = scene.assets[inst.asset]
            sp = a.mlp
            n = a.n
            st = np.zeros(n, np.uint8)
            lg = np.zeros(n)
            mg = np.zeros(n) if want_margin else None
            if sp.kind == 1:
                L.orc_cquery(n, np.ascontiguousarray(a.mean), embeds[inst.asset], inst_array(inst), ca,
                             params64[inst.asset], sp.mean_scale, sp.train_focal, sp.d_min, sp.d_max,
                             int(use_mlp), st, lg, _ptr(mg))
            else:
                L.orc_query(n, np.ascontiguousarray(a.mean), inst_array(inst), ca, params64[inst.asset],
                            sp.width, sp.bands, sp.mean_scale, sp.cam_scale, sp.train_focal, sp.d_min,
                            sp.d_max, int(use_mlp), st, lg, _ptr(mg))
            state[k, off[i]:off[i + 1]] = st
            logit[k, off[i]:off[i + 1]] = lg
            if want_margin:
                margin[k, off[i]:off[i + 1]] = mg
    return (state, logit, margin) if want_margin else (state, logit)


# ----------------------------------------------------------------------------
# the compact MLP form (Sec. 3.2, 3.3, 4.1)
# ----------------------------------------------------------------------------
def cembed(asset):
    """Embeddings [n, 6] of every Gaussian from the asset's embedding MLP, and
    the embedding inputs [n, 8] (opacity, log scales, unit quaternion w >= 0)."""
    n = asset.n
    E = np.zeros((n, 6))
    XE = np.zeros((n, 8))
    lib().orc_cembed(n, np.ascontiguousarray(asset.scale), np.ascontiguousarray(asset.quat),
                     np.ascontiguousarray(asset.opacity), _f64(asset.mlp.params), E, _ptr(XE))
    return E, XE


def cinputs(asset, inst, cam, gidx, E=None):
    """The 16 visibility inputs [m, 16] of Gaussians gidx under an instance and camera."""
    if E is None:
        E = cembed(asset)[0]
    gidx = np.ascontiguousarray(gidx, np.int64)
    X = np.zeros((len(gidx), 16))
    sp = asset.mlp
    lib().orc_cinputs(len(gidx), gidx, asset.n, np.ascontiguousarray(asset.mean), np.ascontiguousarray(E),
                      inst_array(inst), cam_array(cam), sp.train_focal, sp.d_min, sp.d_max, sp.mean_scale, X)
    return X


def cmlp_forward(params, X):
    """Logits and the sum |wo h2| + |bo| of the compact visibility MLP."""
    X = _f64(X)
    z = np.zeros(X.shape[0])
    sc = np.zeros(X.shape[0])
    lib().orc_cmlp_forward(_f64(params), X, X.shape[0], z, _ptr(sc))
    return z, sc


def cjoint_forward(params, XV, XE):
    """Logits and term sizes of the joint compact model (embedding MLP, then
    the visibility MLP) on raw inputs XV [B, 10] and XE [B, 8]."""
    XV, XE = _f64(XV), _f64(XE)
    z = np.zeros(XV.shape[0])
    sc = np.zeros(XV.shape[0])
    lib().orc_cjoint_forward(_f64(params), XV, XE, XV.shape[0], z, _ptr(sc))
    return z, sc


def cmlp_forward_bf16(params, X):
    """Logits of the compact visibility MLP with its second-layer operands
    rounded to BF16 (the reduced-precision form of the query)."""
    X = _f64(X)
    z = np.zeros(X.shape[0])
    lib().orc_cmlp_forward_bf16(_f64(params), X, X.shape[0], z)
    return z


def cbce_backward(params, XV, XE, y, w=None):
    """Mean (weighted) BCE of the joint compact model and its gradient over all
    parameters (visibility, then embedding)."""
    B = len(y)
    dP = np.zeros(lib().orc_compact_sizes(0) + lib().orc_compact_sizes(1))
    loss = lib().orc_cbce_backward(_f64(params), _f64(XV), _f64(XE), _f64(y), _ptr(_f64(w) if w is not None else None),
                                   B, dP)
    return loss, dP


def compact(state: np.ndarray) -> List[np.ndarray]:
    """Compaction: per camera, the kept pair indices in increasing (instance, Gaussian)
    order; the splat id is the running index over cameras."""
    return [np.flatnonzero(state[k] == 2).astype(np.int64) for k in range(state.shape[0])]


def pair_to_instance(scene, pairs: np.ndarray):
    off = scene.pair_offsets()
    inst = np.searchsorted(off, pairs, side="right") - 1
    return inst.astype(np.int64), (pairs - off[inst]).astype(np.int64)


def project(scene, cam, pairs: np.ndarray, det_clip: float = 0.0):
    """Projection + footprint for the kept pairs of one camera, in the given
    order.  det_clip > 0: radius clipping (Sec. 4.3 ablation), a splat whose
    2D covariance (dilated) has determinant below det_clip gets no footprint."""
    inst_of, g_of = pair_to_instance(scene, pairs)
    m = len(pairs)
    rec = np.zeros((m, REC))
    prect = np.zeros((m, 4), np.int32)
    L = lib()
    ca = cam_array(cam)
    for i in np.unique(inst_of):
        sel = np.flatnonzero(inst_of == i)
        inst = scene.instances[int(i)]
        a = scene.assets[inst.asset]
        r = np.zeros((len(sel), REC))
        pr = np.zeros((len(sel), 4), np.int32)
        L.orc_project(len(sel), np.ascontiguousarray(g_of[sel]), a.n, np.ascontiguousarray(a.mean),
                      np.ascontiguousarray(a.scale), np.ascontiguousarray(a.quat),
                      np.ascontiguousarray(a.opacity), np.ascontiguousarray(a.sh), a.sh_degree,
                      inst_array(inst), ca, r, pr)
        rec[sel] = r
        prect[sel] = pr
    if det_clip > 0.0:
        det = rec[:, 2] * rec[:, 4] - rec[:, 3] ** 2  # A C - B^2 of the dilated 2D covariance
        prect[det < det_clip] = (1, 0, 1, 0)
    return rec, prect


def render_camera(rec, prect, cam, tile: int, bg=(0.0, 0.0, 0.0), contrib=None, reached=None,
                  want_margin: bool = True, want_order: bool = False, smargin=None):
    """Binning + compositing for one camera.  contrib/reached arrays (length m) and
    smargin [m, 2] (per-splat decision margins, min-accumulated; start at inf) are
    updated in place when given."""
    m = rec.shape[0]
    H, W = cam.height, cam.width
    img = np.zeros((H, W, 3))
    tf = np.zeros((H, W))
    mg = np.zeros((H, W, 2)) if want_margin else None
    cap = 0
    order = None
    if want_order:
        cap = int(np.sum(_tiles_per_rect(prect, tile))) if m else 0
        order = np.zeros((max(cap, 1), 2), np.int64)
    n = lib().orc_render(m, _f64(rec), np.ascontiguousarray(prect, np.int32), cam_array(cam), tile,
                         _f64(bg), img, _ptr(tf), _ptr(contrib), _ptr(reached), _ptr(mg), _ptr(order), cap,
                         _ptr(smargin))
    out = {"image": img, "T": tf, "entries": int(n)}
    if want_margin:
        out["margin"] = mg
    if want_order:
        out["order"] = order[:n]
    return out


def render_brute(rec, cam, bg=(0.0, 0.0, 0.0)):
    H, W = cam.height, cam.width
    img = np.zeros((H, W, 3))
    tf = np.zeros((H, W))
    lib().orc_render_brute(rec.shape[0], _f64(rec), cam_array(cam), _f64(bg), img, _ptr(tf))
    return img, tf


def _tiles_per_rect(prect, tile):
    pr = np.asarray(prect, np.int64)
    empty = (pr[:, 0] > pr[:, 1]) | (pr[:, 2] > pr[:, 3])
    nx = pr[:, 1] // tile - pr[:, 0] // tile + 1
    ny = pr[:, 3] // tile - pr[:, 2] // tile + 1
    return np.where(empty, 0, nx * ny)


def frame(scene, use_mlp: bool = True, tile: Optional[int] = None, record: bool = False,
          want_margin: bool = True):
    """The whole per-frame path for every camera of the scene."""
    tile = scene.tile if tile is None else tile
    state, logit = query(scene, use_mlp=use_mlp)
    kept = compact(state)
    out = {"state": state, "logit": logit, "kept": kept, "images": [], "T": [], "margin": [],
           "rec": [], "prect": [], "contrib": [], "reached": [], "entries": []}
    for k, cam in enumerate(scene.cameras):
        rec, prect = project(scene, cam, kept[k])
        cb = np.zeros(len(kept[k])) if record else None
        rc = np.zeros(len(kept[k]), np.uint8) if record else None
        r = render_camera(rec, prect, cam, tile, scene.bg, cb, rc, want_margin=want_margin)
        out["images"].append(r["image"])
        out["T"].append(r["T"])
        out["margin"].append(r.get("margin"))
        out["rec"].append(rec)
        out["prect"].append(prect)
        out["contrib"].append(cb)
        out["reached"].append(rc)
        out["entries"].append(r["entries"])
    return out


def contributions(asset, views, tile: int = 16, want_detail: bool = False):
    """Largest contribution alpha*T of each Gaussian's blended fragments in
    each view (Sec. 3.1), single identity instance, frustum culling only:
    [V, n] (0 where outside the frustum or never blended).  want_detail: also
    the "reached" flags [V, n] and the per-Gaussian decision margins
    [V, n, 2] (inf where never tested)."""
    from synth import Scene, identity_instance  # inputs only
    sc = Scene(assets=[asset], instances=[identity_instance(0)], cameras=list(views), tile=tile)
    state, _ = query(sc, use_mlp=False)
    kept = compact(state)
    out = np.zeros((len(views), asset.n))
    rch = np.zeros((len(views), asset.n), np.uint8)
    smg = np.full((len(views), asset.n, 2), np.inf)
    for k, cam in enumerate(views):
        rec, prect = project(sc, cam, kept[k])
        cb = np.zeros(len(kept[k]))
        rc = np.zeros(len(kept[k]), np.uint8)
        sm = np.full((len(kept[k]), 2), np.inf)
        render_camera(rec, prect, cam, tile, (0.0, 0.0, 0.0), cb, rc if want_detail else None,
                      want_margin=False, smargin=sm if want_detail else None)
        out[k, kept[k]] = cb
        rch[k, kept[k]] = rc
        smg[k, kept[k]] = sm
    return (out, rch, smg) if want_detail else out


def aux_views(view, aux: int, angle: float):
    """Auxiliary views (Sec. 3.1): the camera turned rigidly about the asset
    centre by `angle` so that it stays at its distance on the cone around its
    direction d, at `aux` evenly spaced azimuths phi_j = 2 pi j / aux measured
    from e1 = the camera's right axis made orthogonal to d (e2 = d x e1).
    Position and orientation are rotated by the same rotation matrix."""
    from synth import Camera  # inputs only
    if aux == 0:
        return []
    pos = np.asarray(view.pos, np.float64)
    d = pos / np.linalg.norm(pos)
    Rc = np.asarray(view.R, np.float64).reshape(3, 3)
    e1 = Rc[0] - np.dot(Rc[0], d) * d
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    out = []
    for j in range(aux):
        phi = 2.0 * math.pi * j / aux
        k = math.cos(phi) * e1 + math.sin(phi) * e2
        K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
        M = np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)  # rotation by angle about k
        out.append(Camera(pos=(M @ pos).astype(np.float32), R=(Rc @ M.T).astype(np.float32), fovy=view.fovy,
                          width=view.width, height=view.height, near=view.near))
    return out


def labels(asset, views, threshold: float = 1.0 / 255.0, tile: int = 16, aux: int = 0,
           aux_angle: float = 0.0) -> np.ndarray:
    """Labels (Sec. 3.1): label[v, g] = 1 iff Gaussian g's largest contribution
    alpha*T over the pixels of view v, or of one of its auxiliary views,
    exceeds the threshold."""
    out = np.zeros((len(views), asset.n), np.uint8)
    for k, v in enumerate(views):
        group = [v] + aux_views(v, aux, aux_angle)
        out[k] = np.any(contributions(asset, group, tile) > threshold, axis=0)
    return out


def sample_pairs(seed: int, step: int, batch: int, n: int, V: int):
    """(Gaussian, view) pairs of one training step, drawn with SplitMix64 at
    counter step * batch + i: g = (low32(r) n) >> 32, v = (high32(r) V) >> 32."""
    L = lib()
    g = np.zeros(batch, np.int64)
    v = np.zeros(batch, np.int64)
    for i in range(batch):
        r = int(L.orc_splitmix64(seed, step * batch + i))
        g[i] = ((r & 0xFFFFFFFF) * n) >> 32
        v[i] = ((r >> 32) * V) >> 32
    return g, v


# ----------------------------------------------------------------------------
# metrics
# ----------------------------------------------------------------------------
def psnr(a: np.ndarray, b: np.ndarray, cap: float = 100.0) -> float:
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    if mse == 0.0:
        return cap
    return min(cap, 10.0 * math.log10(1.0 / mse))


def flip_rate(keep_a: np.ndarray, keep_b: np.ndarray, in_frustum: np.ndarray) -> float:
    n = int(np.sum(in_frustum))
    if n == 0:
        return 0.0
    return float(np.sum((keep_a != keep_b) & in_frustum)) / n
