"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Protocol for discrete decisions (FP32 kernels vs FP64 oracle):
 (i) same input: the oracle's decision rule applied to the kernel's own FP32
     upstream values must reproduce the kernel's output exactly;
 (ii) from scratch: decisions must agree except where the FP64 decision margin
     is below a small relative threshold (counted and bounded).
Pixels must be within 1e-4 unless a decision on that pixel was within margin.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import scenes

pytestmark = pytest.mark.gpu

from tests.protocol import MARGIN, MARGIN_ALPHA, MARGIN_DEPTH, check_pixels, rect_bound_margin  # noqa: F401


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nvgs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_19202_amd as m
    m.lib()
    return m


def make_ctx(nvgs, sc):
    ctx = nvgs.Context(0)
    ctx.load_assets(sc.assets)
    ctx.set_instances(sc.instances)
    return ctx


def logit_tol(z64, scale):
    return 1e-5 * np.maximum(np.abs(z64), scale)


SCENES = {
    "tiny": lambda: scenes.tiny(),
    "tiny_w128": lambda: scenes.tiny(n=5000, res=128, width=128),
    "composed_small": lambda: scenes.composed_small(),
    "batched_small": lambda: scenes.batched_small(),
    "tiny_compact": lambda: scenes.tiny_compact(),
    "batched_compact": lambda: scenes.batched_compact(),
}


def _logit_scale(a, inst, cam, gidx):
    """FP64 size |wo h| + |bo| of the terms of each queried logit."""
    if a.mlp.kind == 1:
        return oracle.cmlp_forward(a.mlp.params, oracle.cinputs(a, inst, cam, gidx))[1]
    cl = oracle.local_camera(inst, cam, a.mlp.train_focal, a.mlp.d_max)
    return oracle.mlp_forward(a.mlp.params, a.mlp.width, oracle.mlp_inputs(a, gidx, cl))[1]


QUERY_CASES = [(name, "fp32") for name in SCENES] + \
    [(name, "fp32s") for name in ("tiny", "tiny_w128", "composed_small", "batched_small")]


@pytest.mark.parametrize("name,prec", QUERY_CASES)
def test_query_state_and_logits(nvgs, name, prec):
    """FP32 logits (FP32 matrix cores, and the split form: three BF16
    products per FP32 product) within 1e-5 of the logit scale of the FP64
    oracle's; keep states exact on the kernel's own logits and from scratch
    up to the decision margin."""
    sc = SCENES[name]()
    log(f"[query] scene={name} precision={prec}")
    ctx = make_ctx(nvgs, sc)
    st, lg = ctx.query_visibility(sc.cameras, precision=prec)
    st = st.cpu().numpy()
    lg = lg.cpu().numpy().astype(np.float64)
    ost, olg, omg = oracle.query(sc, want_margin=True)
    # logits: every pair the oracle queried and the GPU queried
    both = ~np.isnan(olg) & ~np.isnan(lg)
    assert both.sum() > 0.3 * (ost > 0).sum()
    # tolerance with the scale term |wo h3| + |bo| from the oracle's own MLP
    z64 = olg[both]
    scale = np.zeros_like(z64)
    off = sc.pair_offsets()
    idx = np.flatnonzero(both.ravel())
    k_of = idx // st.shape[1]
    p_of = idx % st.shape[1]
    inst_of = np.searchsorted(off, p_of, side="right") - 1
    for k in np.unique(k_of):
        for i in np.unique(inst_of[k_of == k]):
            sel = (inst_of == i) & (k_of == k)
            inst = sc.instances[int(i)]
            scale[sel] = _logit_scale(sc.assets[inst.asset], inst, sc.cameras[int(k)], p_of[sel] - off[i])
    err = np.abs(lg[both] - z64)
    tol = logit_tol(z64, scale)
    log(f"[query] {name} {prec}: queried {both.sum()}, max |dz| {err.max():.3e}, max err/tol {np.max(err / tol):.3f}")
    assert np.all(err <= tol)
    # same input: the keep rule applied to the GPU's logits reproduces its state
    gq = ~np.isnan(lg)
    assert np.array_equal(st[gq] == 2, lg[gq] >= 0)
    assert np.all(st[gq] >= 1)
    # from scratch: states agree except near-threshold pairs
    diff = st != ost
    excused = omg < MARGIN
    log(f"[query] {name}: state mismatches {diff.sum()} (excused by margin {np.sum(diff & excused)})")
    assert np.sum(diff & ~excused) == 0
    assert diff.sum() <= max(2, 1e-5 * st.size)
    ctx.close()


def _render_debug(nvgs, sc, tile, use_mlp=True):
    ctx = make_ctx(nvgs, sc)
    img, stats = ctx.render(sc.cameras, tile=tile, use_mlp=use_mlp, keep_debug=True, stats=True)
    dbg = ctx.debug_buffers()
    st, lg = ctx.query_visibility(sc.cameras)
    out = {"img": img.cpu().numpy().astype(np.float64), "stats": stats, "state": st.cpu().numpy(),
           "logit": lg.cpu().numpy()}
    for k, v in dbg.items():
        out[k] = v.cpu().numpy() if hasattr(v, "cpu") else v
    ctx.close()
    return out


def _same_input_rect(u, v, ex, ey, W, H, T):
    """Footprint rectangle rule applied in float32 to the kernel's own values."""
    f = np.float32
    u, v, ex, ey = (np.asarray(a, np.float32) for a in (u, v, ex, ey))
    wx = f(1e-4) * ex + f(1e-3)
    wy = f(1e-4) * ey + f(1e-3)
    x0 = np.maximum(np.ceil(((u - ex) - f(0.5)) - wx), f(0))
    x1 = np.minimum(np.floor(((u + ex) - f(0.5)) + wx), f(W - 1))
    y0 = np.maximum(np.ceil(((v - ey) - f(0.5)) - wy), f(0))
    y1 = np.minimum(np.floor(((v + ey) - f(0.5)) + wy), f(H - 1))
    empty = (x0 > x1) | (y0 > y1)
    return x0.astype(np.int64) // T, x1.astype(np.int64) // T, y0.astype(np.int64) // T, y1.astype(np.int64) // T, empty


@pytest.mark.parametrize("name,tile", [("tiny", 16), ("tiny", 8), ("composed_small", 16), ("composed_small", 32),
                                       ("tiny_compact", 16)])
def test_frame_stages_against_oracle(nvgs, name, tile):
    sc = SCENES[name]()
    log(f"[frame] scene={name} tile={tile}")
    r = _render_debug(nvgs, sc, tile)
    cam = sc.cameras[0]
    W, H = cam.width, cam.height
    ns = r["n_splats"]
    # --- compaction: kept list equals the ordered survivors of the GPU state
    kept_gpu = r["pair"].astype(np.int64) & 0xFFFFFFFF
    kept_ref = np.flatnonzero(r["state"][0] == 2)
    assert ns == len(kept_ref) and np.array_equal(kept_gpu, kept_ref)
    log(f"[frame] {name}: {ns} splats, {r['n_dup']} tile entries")
    # --- projection vs FP64 oracle on the same kept list
    rec, prect = oracle.project(sc, cam, kept_ref)
    ra, rb, rc = r["rec_a"].astype(np.float64), r["rec_b"].astype(np.float64), r["rec_c"].astype(np.float64)
    rd = r["rec_d"].astype(np.float64)
    # the centre as hi + lo parts, against FP64 (hi alone is the nearest float)
    du = np.abs(ra[:, 0] + rd[:, 0] - rec[:, 0]).max(initial=0.0)
    dv = np.abs(ra[:, 1] + rd[:, 1] - rec[:, 1]).max(initial=0.0)
    log(f"[frame] {name}: centre max err u {du:.2e} px, v {dv:.2e} px")
    assert du < 2e-6 and dv < 2e-6
    np.testing.assert_allclose(ra[:, 0], rec[:, 0], rtol=0, atol=np.spacing(np.float32(W)))  # u (pixels)
    np.testing.assert_allclose(ra[:, 1], rec[:, 1], rtol=0, atol=np.spacing(np.float32(H)))  # v
    np.testing.assert_allclose(rc[:, 1], rec[:, 8], rtol=2e-6)               # depth
    np.testing.assert_allclose(rb[:, 1], rec[:, 9], rtol=0, atol=0)          # opacity
    for gi, oi in [(ra[:, 2], 5), (ra[:, 3], 6), (rb[:, 0], 7)]:             # conic
        scale = np.maximum(np.abs(rec[:, 5]), np.abs(rec[:, 7]))
        assert np.max(np.abs(gi - rec[:, oi]) / scale) < 5e-5
    rgb_g = np.stack([rb[:, 2], rb[:, 3], rc[:, 0]], 1)
    np.testing.assert_allclose(rgb_g, rec[:, 10:13], rtol=0, atol=2e-5)
    # --- footprint rectangles: same input exactly, from scratch up to margins
    rect = r["rect"].astype(np.int64) & 0xFFFFFFFF
    gx0, gy0 = rect[:, 0] & 0xFFFF, rect[:, 0] >> 16
    gx1, gy1 = rect[:, 1] & 0xFFFF, rect[:, 1] >> 16
    gn = rect[:, 3]
    sx0, sx1, sy0, sy1, sempty = _same_input_rect(ra[:, 0], ra[:, 1], rc[:, 2], rc[:, 3], W, H, tile)
    assert np.array_equal(sempty, gn == 0)
    ne = ~sempty
    assert np.array_equal(sx0[ne], gx0[ne]) and np.array_equal(sx1[ne], gx1[ne])
    assert np.array_equal(sy0[ne], gy0[ne]) and np.array_equal(sy1[ne], gy1[ne])
    assert np.array_equal(gn[ne], (gx1 - gx0 + 1)[ne] * (gy1 - gy0 + 1)[ne])
    oempty = (prect[:, 0] > prect[:, 1]) | (prect[:, 2] > prect[:, 3])
    mism = (oempty != (gn == 0))
    both = ~oempty & (gn > 0)
    mism[both] |= (prect[both, 0] // tile != gx0[both]) | (prect[both, 1] // tile != gx1[both]) | \
                   (prect[both, 2] // tile != gy0[both]) | (prect[both, 3] // tile != gy1[both])
    dist, close = rect_bound_margin(rec, W, H)
    log(f"[frame] {name}: rect mismatches vs FP64 {mism.sum()} of {ns}, all with a bound within "
        f"{dist[mism].max(initial=0.0):.1e} px of a pixel line" if mism.any() else
        f"[frame] {name}: rect mismatches vs FP64 0 of {ns}")
    assert not np.any(mism & ~close)
    # --- sort order: the (tile, depth, id) order of the kernel's own keys
    sk = r["sorted_key"].astype(np.int64) & 0xFFFFFFFF
    sid = r["sorted_id"].astype(np.int64) & 0xFFFFFFFF
    tiles_x = r["tiles_x"]
    ent_t, ent_i = [], []
    for j in np.flatnonzero(gn > 0):
        for ty in range(gy0[j], gy1[j] + 1):
            for tx in range(gx0[j], gx1[j] + 1):
                ent_t.append(ty * tiles_x + tx)
                ent_i.append(j)
    ent_t = np.asarray(ent_t, np.int64)
    ent_i = np.asarray(ent_i, np.int64)
    dkey = r["rec_c"][:, 1].view(np.uint32).astype(np.int64)[ent_i]
    order = np.lexsort((ent_i, dkey, ent_t))
    assert len(sk) == len(ent_t)
    assert np.array_equal(sk, ent_t[order]) and np.array_equal(sid, ent_i[order])
    # --- pixels vs the FP64 oracle from scratch
    ref = oracle.render_camera(rec, prect, cam, tile, sc.bg)
    check_pixels(r["img"][0], ref, f"frame {name} T={tile}")


def test_image_independent_of_tile_size_and_deterministic(nvgs):
    """Sequential compositing (no list split): the image is bit-identical for
    tile edges 8, 16 and 32 and across repeated frames.  (8x8 tiles skip the
    splats whose footprint box holds no live pixel; the larger tiles only skip
    8x8 blocks their box misses, so this also checks that the skip is exact.)"""
    sc = SCENES["composed_small"]()
    ctx = make_ctx(nvgs, sc)
    imgs = [ctx.render(sc.cameras, tile=t, split=-1).cpu().numpy() for t in (8, 16, 32)]
    again = ctx.render(sc.cameras, tile=16, split=-1).cpu().numpy()
    ctx.close()
    same = np.array_equal(imgs[0], imgs[1]) and np.array_equal(imgs[1], imgs[2]) and np.array_equal(imgs[1], again)
    assert same, "image depends on the tile size or is not deterministic"


@pytest.mark.parametrize("name,tile", [("tiny", 8), ("composed_small", 16), ("composed_small", 32)])
def test_split_lists_match_sequential_and_oracle(nvgs, name, tile):
    """Long tile lists composited in chunks (forced with 64-entry chunks):
    equal to the sequential composite up to rounding, to the FP64 oracle under
    the pixel protocol, deterministic, and the recorded contributions agree."""
    sc = SCENES[name]()
    ctx = make_ctx(nvgs, sc)
    import torch
    seq = ctx.render(sc.cameras, tile=tile, split=-1).cpu().numpy().astype(np.float64)
    img, stats = ctx.render(sc.cameras, tile=tile, split=64, keep_debug=True, stats=True)
    img = img.cpu().numpy().astype(np.float64)
    again = ctx.render(sc.cameras, tile=tile, split=64).cpu().numpy().astype(np.float64)
    st, _ = ctx.query_visibility(sc.cameras)
    st = st.cpu().numpy()
    P = st.shape[1]
    cb_seq = torch.zeros(P, device="cuda")
    cb_split = torch.zeros(P, device="cuda")
    ctx.render(sc.cameras, tile=tile, split=-1, contrib=cb_seq)
    ctx.render(sc.cameras, tile=tile, split=64, contrib=cb_split)
    cb_seq, cb_split = cb_seq.cpu().numpy(), cb_split.cpu().numpy()
    ctx.close()
    assert np.array_equal(img, again), "split composite not deterministic"
    d_seq = np.abs(img - seq).max()
    cam = sc.cameras[0]
    kept = np.flatnonzero(st[0] == 2)
    rec, prect = oracle.project(sc, cam, kept)
    ref = oracle.render_camera(rec, prect, cam, tile, sc.bg)
    dc = np.abs(cb_split - cb_seq)
    log(f"[split] {name} T={tile}: {stats['duplicates']} entries; max |split - sequential| {d_seq:.2e}; "
        f"contrib max diff {dc.max():.2e}")
    check_pixels(img[0], ref, f"split {name} T={tile}")
    assert d_seq < 1e-5 or np.sum(np.abs(img - seq) > 1e-5) <= max(4, 1e-3 * img[..., 0].size)
    assert np.mean(dc <= 1e-5 * np.maximum(cb_seq, 1e-3)) > 0.999


@pytest.mark.parametrize("tile", [8, 16])
def test_default_chunk_length_follows_the_frame(nvgs, tile):
    """The default compositing chunk length is set by the frame on the device:
    max(256, ceil(entries / D)) with D = 2 x compute units x 2048 / threads
    per compositing work-group; the work items are one per tile list plus
    one per extra chunk, and the image is the sequential one up to rounding
    and, where FP64 decides, the oracle's."""
    import torch
    sc = SCENES["composed_small"]()
    ctx = make_ctx(nvgs, sc)
    img, st = ctx.render(sc.cameras, tile=tile, keep_debug=True, stats=True)
    dbg = ctx.debug_buffers()
    sk = dbg["sorted_key"].cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    lens = np.bincount(sk, minlength=len(sc.cameras) * dbg["tiles_x"] * dbg["tiles_y"])
    seq = ctx.render(sc.cameras, tile=tile, split=-1).cpu().numpy().astype(np.float64)
    img = img.cpu().numpy().astype(np.float64)
    q, _ = ctx.query_visibility(sc.cameras)
    q = q.cpu().numpy()
    ctx.close()
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    D = 2 * n_cu * 2048 // (64 if tile == 8 else 256)
    S = max(256, -(-st["duplicates"] // D))
    items = int(np.sum(np.where(lens > S, -(-lens // S), 1)))
    log(f"[chunks] T={tile}: {st['duplicates']} entries, longest list {lens.max()}, chunk {st['chunk_len']} "
        f"(rule {S}), items {st['blend_items']} (rule {items})")
    assert st["chunk_len"] == S and st["blend_items"] == items
    assert lens.max() > S, "the scene has no list long enough to split"
    assert np.abs(img - seq).max() < 1e-5 or np.sum(np.abs(img - seq) > 1e-5) <= max(4, 1e-3 * img[..., 0].size)
    cam = sc.cameras[0]
    rec, prect = oracle.project(sc, cam, np.flatnonzero(q[0] == 2))
    check_pixels(img[0], oracle.render_camera(rec, prect, cam, tile, sc.bg), f"default chunks T={tile}")


def test_unculled_render_matches_oracle(nvgs):
    sc = SCENES["tiny"]()
    ctx = make_ctx(nvgs, sc)
    img = ctx.render(sc.cameras, tile=16, use_mlp=False).cpu().numpy()[0].astype(np.float64)
    ctx.close()
    ref = oracle.frame(sc, use_mlp=False)
    check_pixels(img, {"image": ref["images"][0], "margin": ref["margin"][0]}, "unculled tiny")


def test_empty_frame_and_invalid_arguments(nvgs):
    sc = SCENES["tiny"]()
    ctx = make_ctx(nvgs, sc)
    back = synth.camera((0.0, 3.0, 0.0), target=(0.0, 6.0, 0.0), width=64, height=48)  # looks away
    img, stats = ctx.render([back], tile=16, bg=(0.25, 0.5, 0.75), stats=True)
    assert stats["kept"] == 0 and stats["duplicates"] == 0
    assert np.allclose(img.cpu().numpy(), np.array([0.25, 0.5, 0.75], np.float32))
    with pytest.raises(nvgs.NvgsError) as e:
        ctx.render([back], tile=12)
    assert e.value.status == nvgs.E_INVALID
    bad = synth.camera((0.0, 3.0, 0.0), width=64, height=48)
    bad.fovy = float("nan")
    with pytest.raises(nvgs.NvgsError):
        ctx.render([bad])
    ctx.close()


@pytest.mark.parametrize("prec,width", [("bf16", 64), ("bf16", 128), ("fp8", 64), ("fp8", 128)])
def test_reduced_precision_mlp(nvgs, prec, width):
    """BF16 / FP8 E4M3 MLP forms: the kernel's logits equal the oracle's
    emulation of the same operand rounding (FP64 otherwise) up to FP32
    accumulation order; the keep flip rate against the FP64 MLP is reported."""
    sc = scenes.tiny(n=6000, res=128, width=width)
    log(f"[prec] {prec} W={width}")
    ctx = make_ctx(nvgs, sc)
    st, lg = ctx.query_visibility(sc.cameras, precision=prec)
    st, lg = st.cpu().numpy()[0], lg.cpu().numpy()[0].astype(np.float64)
    ctx.close()
    ost, olg = oracle.query(sc)
    ost, olg = ost[0], olg[0]
    q = ~np.isnan(olg)
    a = sc.assets[0]
    cl = oracle.local_camera(sc.instances[0], sc.cameras[0], a.mlp.train_focal, a.mlp.d_max)
    X = oracle.mlp_inputs(a, np.flatnonzero(q), cl)
    zq = oracle.mlp_forward_q(a.mlp.params, width, X, prec)
    _, scale = oracle.mlp_forward(a.mlp.params, width, X)
    zg = lg[q]
    err = np.abs(zg - zq)
    rel = err / np.maximum(np.abs(zq), scale)
    flips = np.mean((zg >= 0) != (olg[q] >= 0))
    log(f"[prec] {prec} W={width}: max |z-zq| {err.max():.3e}, max rel {rel.max():.3e}, "
        f"p99.9 rel {np.quantile(rel, 0.999):.3e}, flip rate vs FP64 {flips:.4f}")
    # Most pairs agree to FP32 accumulation order.  An activation whose FP32
    # value (kernel) and FP64 value (emulation) straddle a rounding boundary
    # rounds one unit apart: 2^-8 (BF16) or up to 2^-3 (E4M3) of one of the W
    # terms, i.e. ~2^-3/W of the logit scale for FP8; such pairs are rare.
    assert np.median(rel) < 1e-5
    assert np.quantile(rel, 0.999) < (1e-3 if prec == "bf16" else 5e-3)
    assert rel.max() < (1e-2 if prec == "bf16" else 5e-2)
    assert np.array_equal(st[q] == 2, zg >= 0)
    assert flips < (0.02 if prec == "bf16" else 0.08)


def test_compact_mlp_bf16(nvgs):
    """The compact form with BF16 second-layer operands: logits equal the
    oracle's emulation of that rounding up to FP32 accumulation order; FP8
    is refused for this form."""
    sc = scenes.batched_compact()
    log("[prec] compact bf16")
    ctx = make_ctx(nvgs, sc)
    st, lg = ctx.query_visibility(sc.cameras, precision="bf16")
    st, lg = st.cpu().numpy(), lg.cpu().numpy().astype(np.float64)
    with pytest.raises(nvgs.NvgsError):
        ctx.query_visibility(sc.cameras, precision="fp8")
    with pytest.raises(nvgs.NvgsError):
        ctx.render(sc.cameras, precision="fp8")
    ctx.close()
    ost, olg = oracle.query(sc)
    off = sc.pair_offsets()
    zq, z64, zg, scale = [], [], [], []
    for k, cam in enumerate(sc.cameras):
        for i, inst in enumerate(sc.instances):
            q = np.flatnonzero(~np.isnan(olg[k, off[i]:off[i + 1]]))
            if len(q) == 0:
                continue
            a = sc.assets[inst.asset]
            X = oracle.cinputs(a, inst, cam, q)
            zq.append(oracle.cmlp_forward_bf16(a.mlp.params, X))
            z, s = oracle.cmlp_forward(a.mlp.params, X)
            z64.append(z)
            scale.append(s)
            zg.append(lg[k, off[i] + q])
    zq, z64, zg, scale = map(np.concatenate, (zq, z64, zg, scale))
    rel = np.abs(zg - zq) / np.maximum(np.abs(zq), scale)
    flips = np.mean((zg >= 0) != (z64 >= 0))
    log(f"[prec] compact bf16: {len(zg)} queried, median rel {np.median(rel):.3e}, "
        f"p99.9 rel {np.quantile(rel, 0.999):.3e}, max rel {rel.max():.3e}, flip rate vs FP64 {flips:.4f}")
    # a first-layer activation whose FP32 (kernel) and FP64 (emulation) values
    # straddle a BF16 rounding boundary rounds one unit (2^-8 relative) apart
    assert np.median(rel) < 1e-5
    assert np.quantile(rel, 0.999) < 1e-3
    assert rel.max() < 1e-2
    gq = ~np.isnan(lg)
    assert np.array_equal(st[gq] == 2, lg[gq] >= 0)
    assert flips < 0.02


def test_radius_clipping_matches_oracle(nvgs):
    """Radius clipping by the 2D covariance determinant (Sec. 4.3 ablation):
    the splats the kernel leaves unbinned are those whose FP64 determinant is
    below the threshold (up to a relative margin of 1e-5), and the pixels
    match the oracle's clipped frame under the pixel protocol."""
    sc = SCENES["composed_small"]()
    ctx = make_ctx(nvgs, sc)
    st, _ = ctx.query_visibility(sc.cameras)
    kept = np.flatnonzero(st.cpu().numpy()[0] == 2)
    cam = sc.cameras[0]
    rec0, _ = oracle.project(sc, cam, kept)
    det = rec0[:, 2] * rec0[:, 4] - rec0[:, 3] ** 2
    tau = float(np.quantile(det, 0.4))
    img = ctx.render(sc.cameras, tile=16, det_clip=tau, keep_debug=True)
    dbg = ctx.debug_buffers()
    img = img.cpu().numpy()[0].astype(np.float64)
    gn = dbg["rect"].cpu().numpy().astype(np.int64)[:, 3] & 0xFFFFFFFF
    ctx.close()
    rec, prect = oracle.project(sc, cam, kept, det_clip=tau)
    oempty = (prect[:, 0] > prect[:, 1]) | (prect[:, 2] > prect[:, 3])
    # the FP32 determinant (a sum of non-negative terms) is within a few 1e-7
    # relative of FP64; a clip decision closer than 1e-5 may go either way,
    # as may an empty rectangle whose bound sits on a pixel line
    near = np.abs(det - tau) < 1e-5 * tau
    _, close = rect_bound_margin(rec0, cam.width, cam.height)
    mism = oempty != (gn == 0)
    log(f"[clip] tau {tau:.4g}: oracle clips {np.sum(det < tau)} of {len(det)}, mismatches {mism.sum()} "
        f"(determinant near the threshold {np.sum(mism & near)}, a bound on a pixel line {np.sum(mism & close)})")
    assert np.sum(det < tau) > 0.3 * len(det)
    assert not np.any(mism & ~near & ~close)
    ref = oracle.render_camera(rec, prect, cam, 16, sc.bg)
    check_pixels(img, ref, "radius clipping")
