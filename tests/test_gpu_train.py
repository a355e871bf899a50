"""Differentiation form: the hand-written MLP backward, the autograd
function, renderer-made labels and training, against the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.protocol import MARGIN_ALPHA, MARGIN_DEPTH

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_19202_amd as nvgs
    ctx = nvgs.Context(0)
    yield nvgs, ctx, torch
    ctx.close()


def _batch(B, seed, width=64):
    g = np.random.default_rng(seed)
    p = synth.mlp_params(width, synth.rng(seed)).astype(np.float32)
    X = g.uniform(-1, 1, (B, 72)).astype(np.float32)
    y = (g.uniform(0, 1, B) > 0.5).astype(np.float64)
    return p, X, y


def _grad_close(dg, do, tol=1e-3):
    floor = 1e-6 * np.max(np.abs(do))
    rel = np.abs(dg - do) / np.maximum(np.abs(do), floor)
    return np.linalg.norm(dg - do) / np.linalg.norm(do), rel


@pytest.mark.parametrize("width,B", [(64, 300), (64, 1024), (64, 65536), (128, 300), (128, 1024), (128, 4133)])
def test_mlp_forward_backward_fp32_vs_oracle(env, width, B):
    """FP32 forward and hand-written backward against the FP64 oracle at both
    widths (65,536: the differentiation workload's batch; 4,133: several
    work-groups and a ragged last chunk at width 128)."""
    nvgs, ctx, torch = env
    p, X, y = _batch(B, 5 + B, width)
    z64, scale = oracle.mlp_forward(p, width, X)
    zg = ctx.mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    err = np.abs(zg - z64) / (1e-5 * np.maximum(np.abs(z64), scale))
    log(f"[grad] W={width} B={B}: logits max err/tol {err.max():.3f}")
    assert np.all(err <= 1.0)
    dlog = ((1 / (1 + np.exp(-z64)) - y) / B).astype(np.float32)
    loss, dP, dX = oracle.bce_backward(p, width, X, y, want_dx=True)
    dp_g, dx_g = ctx.mlp_backward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(), torch.from_numpy(dlog).cuda())
    nrm, rel = _grad_close(dp_g.cpu().numpy().astype(np.float64), dP)
    log(f"[grad] W={width} B={B}: param grad rel norm err {nrm:.2e}, max rel {rel.max():.2e}")
    assert nrm < 1e-3 and np.mean(rel < 1e-3) > 0.999
    nrm_x, rel_x = _grad_close(dx_g.cpu().numpy().astype(np.float64), dX)
    log(f"[grad] W={width} B={B}: input grad rel norm err {nrm_x:.2e}")
    assert nrm_x < 1e-3


@pytest.mark.parametrize("width", [64, 128])
def test_mlp_backward_bf16_cosine(env, width):
    """The BF16 form (BF16 matrix-core GEMMs, FP32 accumulation): logits near
    FP64's, and the parameter gradient points the FP64 way (cosine >= 0.999).
    The input gradient's last product has BF16 operands on both sides and no
    sum over the batch to average their rounding, so it is held to 0.99."""
    nvgs, ctx, torch = env
    B = 2048
    p, X, y = _batch(B, 9, width)
    z64, scale = oracle.mlp_forward(p, width, X)
    zb = ctx.mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(), precision="bf16").cpu().numpy()
    zerr = np.abs(zb - z64) / scale  # BF16 operands: about 2^-9 relative each
    log(f"[grad] W={width} bf16 logits vs FP64: error / logit scale median {np.median(zerr):.2e}, "
        f"max {zerr.max():.2e}")
    assert np.median(zerr) < 5e-3 and zerr.max() < 5e-2
    dlog = ((1 / (1 + np.exp(-z64)) - y) / B).astype(np.float32)
    _, dP, dX = oracle.bce_backward(p, width, X, y, want_dx=True)
    dp_g, dx_g = ctx.mlp_backward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(),
                                  torch.from_numpy(dlog).cuda(), precision="bf16")
    g = dp_g.cpu().numpy().astype(np.float64)
    cos = float(np.dot(g, dP) / (np.linalg.norm(g) * np.linalg.norm(dP)))
    gx = dx_g.cpu().numpy().astype(np.float64).ravel()
    cos_x = float(np.dot(gx, dX.ravel()) / (np.linalg.norm(gx) * np.linalg.norm(dX)))
    log(f"[grad] W={width} bf16 cosine similarity to the FP64 gradient: params {cos:.6f}, inputs {cos_x:.6f}")
    assert cos >= 0.999 and cos_x >= 0.99


def test_autograd_function(env):
    nvgs, ctx, torch = env
    B = 512
    p, X, y = _batch(B, 13)
    Xt = torch.from_numpy(X).cuda().requires_grad_(True)
    pt = torch.from_numpy(p).cuda().requires_grad_(True)
    f = nvgs.visibility_mlp_function()
    z = f.apply(Xt, pt, ctx, "fp32")
    loss = torch.nn.functional.binary_cross_entropy_with_logits(z, torch.from_numpy(y).float().cuda())
    loss.backward()
    l64, dP, dX = oracle.bce_backward(p, 64, X, y, want_dx=True)
    assert abs(loss.item() - l64) < 1e-5
    assert _grad_close(pt.grad.cpu().numpy().astype(np.float64), dP)[0] < 1e-3
    assert _grad_close(Xt.grad.cpu().numpy().astype(np.float64), dX)[0] < 1e-3


def _small_asset(n=3000, seed=4, width=64):
    a = synth.make_asset("torus", n, 0, seed, width=width, cam_scale=1.0 / 20.0, d_max=20.0)
    a.opacity[:] = np.clip(a.opacity * 1.2, 0, 1)
    a.scale[:] *= 2.0
    return a


def _label_bits(lab, V, n):
    return np.unpackbits(lab.view(np.uint8).reshape(V, -1), axis=1, bitorder="little")[:, :n].astype(bool)


def _label_excusal(cb, smg):
    """Label decisions the FP32 renderer may take differently from FP64: the
    contribution itself within MARGIN_ALPHA (relative) of 1/255, or a decision
    that shapes it (an alpha or stop test, the depth order of two fragments)
    within margin at a pixel where the Gaussian was tested or listed after a
    stop.  cb [V, n], smg [V, n, 2] from the oracle."""
    near = np.abs(cb - 1 / 255) < MARGIN_ALPHA / 255
    return near | (smg[..., 0] < MARGIN_ALPHA) | (smg[..., 1] < MARGIN_DEPTH)


def _check_labels(bits, cb, smg, label):
    ref = cb > 1 / 255
    diff = bits != ref
    exc = _label_excusal(cb, smg)
    log(f"[labels {label}] {ref.mean():.3f} visible; mismatches {diff.sum()} of {diff.size} "
        f"(excused: contribution near 1/255 {np.sum(diff & (np.abs(cb - 1 / 255) < MARGIN_ALPHA / 255))}, "
        f"a decision in margin {np.sum(diff & exc)})")
    assert not np.any(diff & ~exc)
    return ref


@pytest.mark.parametrize("aux", [0, 6])
def test_labels_match_oracle(env, aux):
    """Labels rendered by the library equal the oracle's (largest alpha*T over
    the view and its auxiliary views above 1/255) except where a decision that
    shapes the contribution is within the FP32 margin."""
    nvgs, ctx, torch = env
    a = _small_asset()
    views = synth.label_views(6, seed=3, d_lo=2.0, d_hi=4.0, res=96, offset=0.2)
    ang = math.radians(5.0)
    ctx.load_assets([a])
    lab = ctx.make_labels(0, views, aux=aux, aux_angle=ang).cpu().numpy().view(np.uint32)
    bits = _label_bits(lab, len(views), a.n)
    cb, smg = [], []
    for v in views:
        c, _, m = oracle.contributions(a, [v] + oracle.aux_views(v, aux, ang), want_detail=True)
        cb.append(c.max(axis=0))
        smg.append(m.min(axis=0))
    ref = _check_labels(bits, np.stack(cb), np.stack(smg), f"aux={aux}")
    assert 0.1 < ref.mean() < 0.95


def test_labels_full_size(env):
    """Labels of the differentiation workload's own asset (500k SH3
    Gaussians) on three of its 512 label views at 512x512, against the
    oracle's largest alpha*T per Gaussian, under the same margin rule."""
    nvgs, ctx, torch = env
    sc = synth.scene_train()
    a = sc.assets[0]
    views = synth.label_views(512, seed=synth.SEED_BASE + 5, d_lo=1.5, d_hi=20.0, res=512)
    views = [views[j] for j in (0, 171, 342)]
    ctx.load_assets([a])
    lab = ctx.make_labels(0, views).cpu().numpy().view(np.uint32)
    bits = _label_bits(lab, len(views), a.n)
    cb, _, smg = oracle.contributions(a, views, want_detail=True)
    ref = _check_labels(bits, cb, smg, f"full size {a.n} x {len(views)}")
    assert 0.01 < ref.mean() < 0.95


def test_labels_same_input(env):
    """Same input: label bits recomputed on the host from the renderer's own
    recorded contributions (frames of the same views, tile and chunking)
    equal the library's label bits exactly."""
    nvgs, ctx, torch = env
    a = _small_asset(n=20000, seed=8)
    views = synth.label_views(12, seed=9, d_lo=1.5, d_hi=6.0, res=128, offset=0.2)
    ctx.load_assets([a])
    lab = ctx.make_labels(0, views, tile=16).cpu().numpy().view(np.uint32)
    bits = _label_bits(lab, len(views), a.n)
    ctx.set_instances([synth.identity_instance(0)])
    cb = torch.zeros((len(views), a.n), device="cuda")
    ctx.render(views, tile=16, use_mlp=False, contrib=cb)
    cb = cb.cpu().numpy()
    host = cb > np.float32(1 / 255)
    log(f"[labels same input] {host.mean():.3f} visible, {np.sum(bits != host)} differences")
    assert np.array_equal(bits, host)


def test_reached_and_ground_truth_visibility(env):
    """Contributions and "reached" flags (contrib > 0) of a frame against the
    oracle's, under the margin rule; then the ground-truth-visibility
    invariant on the GPU: removing every pair the renderer never reached
    (contrib == 0: skipped wherever tested, or listed after the stop) leaves
    every pixel bit-identical, and removing every pair it never blended (also
    the fragments that stopped a pixel) changes no pixel by more than that
    pixel's transmittance at the stop (T_final, read as the difference of a
    white- and a black-background frame) times the largest colour."""
    nvgs, ctx, torch = env
    a = _small_asset(n=20000, seed=10)
    cam = synth.label_views(1, seed=12, d_lo=2.5, d_hi=2.5, res=128)[0]
    ctx.load_assets([a])
    ctx.set_instances([synth.identity_instance(0)])
    cb = torch.zeros(a.n, device="cuda")
    img = ctx.render([cam], tile=16, use_mlp=False, contrib=cb, split=-1).cpu().numpy()[0]
    white = ctx.render([cam], tile=16, use_mlp=False, bg=(1.0, 1.0, 1.0), split=-1).cpu().numpy()[0]
    cb = cb.cpu().numpy()
    reached_g = cb > 0
    c64, r64, smg = oracle.contributions(a, [cam], want_detail=True)
    exc = (smg[0, :, 0] < MARGIN_ALPHA) | (smg[0, :, 1] < MARGIN_DEPTH)
    dr = reached_g != r64[0].astype(bool)
    log(f"[reached] GPU {reached_g.sum()}, oracle {int(r64.sum())} of {a.n}; mismatches {dr.sum()} "
        f"(excused {np.sum(dr & exc)})")
    assert not np.any(dr & ~exc)
    blended = cb >= np.finfo(np.float32).tiny
    both = blended & (c64[0] > 0) & ~exc
    rel = np.abs(cb[both] - c64[0][both]) / c64[0][both]
    log(f"[reached] contributions of {both.sum()} blended pairs: max rel err {rel.max():.2e}")
    assert rel.max() < MARGIN_ALPHA
    assert reached_g.sum() > blended.sum() > 0.2 * a.n  # some pairs stop a pixel without blending

    def without(keep):
        b = synth.Asset(mean=a.mean, scale=a.scale, quat=a.quat, opacity=np.where(keep, a.opacity, 0).astype(np.float32),
                        sh=a.sh, sh_degree=a.sh_degree, mlp=a.mlp)
        ctx.load_assets([b])
        ctx.set_instances([synth.identity_instance(0)])
        return ctx.render([cam], tile=16, use_mlp=False, split=-1).cpu().numpy()[0]

    img_r = without(reached_g)
    log(f"[ground truth] removing {np.sum(~reached_g)} never-reached pairs: max change {np.abs(img_r - img).max():.2e}")
    assert np.array_equal(img_r, img)
    img_b = without(blended)
    t_final = (white - img)[..., 0]
    bound = t_final * _max_colour(a, cam)
    dch = np.abs(img_b - img).max(axis=2)
    log(f"[ground truth] removing {np.sum(~blended)} never-blended pairs: max change {dch.max():.2e}, "
        f"{np.sum(dch > 1e-4)} pixels above 1e-4 (each within its T at the stop: worst ratio "
        f"{np.max(dch / np.maximum(bound, 1e-30)):.3f})")
    assert np.all(dch <= bound + 1e-6)
    ctx.load_assets([a])


def _max_colour(a, cam):
    """Largest colour channel of the asset's in-frustum Gaussians seen from
    cam (the oracle's SH colour, an upper bound per fragment)."""
    sc = synth.Scene(assets=[a], instances=[synth.identity_instance(0)], cameras=[cam], tile=16)
    st, _ = oracle.query(sc, use_mlp=False)
    rec, _ = oracle.project(sc, cam, np.flatnonzero(st[0] == 2))
    return float(rec[:, 10:13].max())


@pytest.mark.parametrize("weighting,width", [(0, 64), (1, 64), (1, 128)])
def test_training_step_matches_oracle(env, weighting, width):
    """One FP32 Adam step on oracle labels: the GPU's batch loss equals the
    oracle's on the same SplitMix64-drawn pairs, and the first Adam update
    (lr * sign(g) where |g| >> eps) agrees."""
    nvgs, ctx, torch = env
    a = _small_asset(n=2000, seed=6, width=width)
    views = synth.label_views(4, seed=5, d_lo=2.0, d_hi=4.0, res=64)
    lab = oracle.labels(a, views)
    words = (a.n + 31) // 32
    packed = np.zeros((len(views), words * 32), np.uint8)
    packed[:, :a.n] = lab
    lab_words = np.packbits(packed, axis=1, bitorder="little").view(np.uint32).reshape(len(views), words)
    ctx.load_assets([a])
    p0 = a.mlp.params.astype(np.float32)
    pt = torch.from_numpy(p0.copy()).cuda()
    B, seed, lr = 1000, 77, 1e-3
    curve = ctx.train_visibility(0, views, pt, labels=torch.from_numpy(lab_words.view(np.int32)).cuda(), batch=B,
                                 steps=1, precision="fp32", lr=lr, seed=seed, weighting=weighting)
    g_idx, v_idx = oracle.sample_pairs(seed, 0, B, a.n, len(views))
    X = np.zeros((B, 72))
    for v in np.unique(v_idx):
        sel = np.flatnonzero(v_idx == v)
        cl = oracle.local_camera(synth.identity_instance(), views[v], a.mlp.train_focal, a.mlp.d_max)
        X[sel] = oracle.mlp_inputs(a, g_idx[sel], cl)
    y = lab[v_idx, g_idx].astype(np.float64)
    w = None
    if weighting:  # each sample weighted by B / (2 n_class)
        npos = y.sum()
        w = np.where(y > 0.5, B / (2 * npos), B / (2 * (B - npos)))
    loss, dP = oracle.bce_backward(p0, width, X, y, w=w)
    log(f"[train] W={width}: loss gpu {curve[0]:.6f} oracle {loss:.6f}")
    assert abs(curve[0] - loss) < 1e-5 * max(1.0, loss)
    p64 = p0.astype(np.float64)
    m = np.zeros_like(p64); v = np.zeros_like(p64)
    oracle.adam_step(p64, dP, m, v, 1, lr=lr)
    dg = pt.cpu().numpy().astype(np.float64) - p0
    do = p64 - p0
    big = np.abs(dP) > 1e-5 * np.abs(dP).max()
    agree = np.abs(dg - do) < 1e-6
    log(f"[train] first update agrees on {agree[big].mean():.5f} of {big.sum()} parameters")
    assert agree[big].mean() > 0.995


def _oracle_inputs(a, views, g_idx, v_idx):
    X = np.zeros((len(g_idx), 72))
    for v in np.unique(v_idx):
        sel = np.flatnonzero(v_idx == v)
        cl = oracle.local_camera(synth.identity_instance(), views[v], a.mlp.train_focal, a.mlp.d_max)
        X[sel] = oracle.mlp_inputs(a, g_idx[sel], cl)
    return X


def test_training_schedule_matches_oracle(env):
    """The warm-up + exponential-decay schedule (Sec. 4.1) in training: four
    FP32 steps with lr_final > 0 against the oracle's Adam run with the
    oracle's schedule on the same SplitMix64 pairs (the learning rate of each
    step scales its update, so a rate off by a step or a factor shows)."""
    nvgs, ctx, torch = env
    a = _small_asset(n=2000, seed=6)
    views = synth.label_views(4, seed=5, d_lo=2.0, d_hi=4.0, res=64)
    lab = oracle.labels(a, views)
    words = (a.n + 31) // 32
    packed = np.zeros((len(views), words * 32), np.uint8)
    packed[:, :a.n] = lab
    lab_words = np.packbits(packed, axis=1, bitorder="little").view(np.uint32).reshape(len(views), words)
    ctx.load_assets([a])
    p0 = a.mlp.params.astype(np.float32)
    steps, B, seed, lr, lr_final = 10, 1000, 91, 2e-3, 2e-4
    p64 = p0.astype(np.float64)
    m = np.zeros_like(p64); v = np.zeros_like(p64)
    rates = [oracle.lr_schedule(lr, lr_final, steps, t) for t in range(steps)]
    for t in range(steps):
        g_idx, v_idx = oracle.sample_pairs(seed, t, B, a.n, len(views))
        X = _oracle_inputs(a, views, g_idx, v_idx)
        _, dP = oracle.bce_backward(p64, 64, X, lab[v_idx, g_idx].astype(np.float64))
        oracle.adam_step(p64, dP, m, v, t + 1, lr=rates[t])
    pt = torch.from_numpy(p0.copy()).cuda()
    ctx.train_visibility(0, views, pt, labels=torch.from_numpy(lab_words.view(np.int32)).cuda(), batch=B,
                         steps=steps, precision="fp32", lr=lr, seed=seed, lr_final=lr_final)
    dg = pt.cpu().numpy().astype(np.float64) - p0
    do = p64 - p0
    big = np.abs(do) > 0.5 * sum(rates)  # parameters whose updates kept one sign
    rel = np.abs(dg - do) / np.abs(do)
    log(f"[schedule] rates {['%.3g' % r for r in rates]}; {big.sum()} steadily moving parameters, "
        f"update rel err median {np.median(rel[big]):.2e}, within 1e-3: {np.mean(rel[big] < 1e-3):.4f}")
    assert rates[0] < rates[1] and rates[-1] == pytest.approx(lr_final, rel=1e-6)
    assert big.sum() > 100 and np.mean(rel[big] < 1e-3) > 0.99


@pytest.mark.parametrize("width", [64, 128])
def test_training_reduces_loss(env, width):
    nvgs, ctx, torch = env
    a = _small_asset(n=4000, seed=8, width=width)
    views = synth.label_views(24, seed=9, d_lo=2.0, d_hi=6.0, res=96)
    ctx.load_assets([a])
    pt = torch.from_numpy(a.mlp.params.astype(np.float32).copy()).cuda()
    curve = ctx.train_visibility(0, views, pt, batch=4096, steps=300, precision="bf16", lr=3e-3, seed=1)
    log(f"[train] W={width}: loss {curve[0]:.4f} -> {curve[-20:].mean():.4f}")
    assert np.all(np.isfinite(curve))
    assert curve[-20:].mean() < 0.8 * curve[:5].mean()


# ---------------------------------------------------------------------------
# the compact form (Sec. 3.2, 3.3, 4.1): embedding and visibility MLPs jointly
# ---------------------------------------------------------------------------
def _compact_batch(B, seed):
    """Raw inputs of the joint model: ten visibility inputs (normalised mean,
    unit direction, distance in [-1, 1], unit forward vector) and eight
    embedding inputs (opacity, log scales, unit quaternion with w >= 0)."""
    g = np.random.default_rng(seed)
    p = synth.compact_params(g)
    unit = lambda m: m / np.linalg.norm(m, axis=1, keepdims=True)
    XV = np.concatenate([g.uniform(-1, 1, (B, 3)), unit(g.standard_normal((B, 3))), g.uniform(-1, 1, (B, 1)),
                         unit(g.standard_normal((B, 3)))], 1)
    q = unit(g.standard_normal((B, 4)))
    q *= np.where(q[:, :1] < 0, -1.0, 1.0)
    XE = np.concatenate([g.uniform(0.3, 1, (B, 1)), g.normal(-4.5, 0.3, (B, 3)), q], 1)
    X = np.concatenate([XV, XE], 1).astype(np.float32)
    y = (g.uniform(0, 1, B) > 0.5).astype(np.float64)
    return p, X, y


@pytest.mark.parametrize("B", [300, 1024, 70000])
def test_compact_forward_backward_fp32_vs_oracle(env, B):
    nvgs, ctx, torch = env
    p, X, y = _compact_batch(B, 30 + B)
    XV, XE = X[:, :10].astype(np.float64), X[:, 10:].astype(np.float64)
    z64, scale = oracle.cjoint_forward(p, XV, XE)
    pt, Xt = torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda()
    zg = ctx.cmlp_forward(pt, Xt).cpu().numpy().astype(np.float64)
    err = np.abs(zg - z64) / np.maximum(np.abs(z64), scale)
    log(f"[cgrad] B={B}: forward max err / max(|z|, scale) {err.max():.2e}")
    assert err.max() < 1e-5
    dlog = ((1 / (1 + np.exp(-z64)) - y) / B).astype(np.float32)
    _, dP = oracle.cbce_backward(p, XV, XE, y)
    dg = ctx.cmlp_backward(pt, Xt, torch.from_numpy(dlog).cuda()).cpu().numpy().astype(np.float64)
    nrm, rel = _grad_close(dg, dP)
    nv = synth.COMPACT_VIS_PARAMS
    log(f"[cgrad] B={B}: param grad rel norm err {nrm:.2e} (visibility "
        f"{np.linalg.norm(dg[:nv] - dP[:nv]) / np.linalg.norm(dP[:nv]):.2e}, embedding "
        f"{np.linalg.norm(dg[nv:] - dP[nv:]) / np.linalg.norm(dP[nv:]):.2e}), max rel {rel.max():.2e}")
    assert nrm < 1e-4 and np.mean(rel < 1e-3) > 0.999


def test_compact_backward_bf16_and_autograd(env):
    nvgs, ctx, torch = env
    B = 4096
    p, X, y = _compact_batch(B, 77)
    XV, XE = X[:, :10].astype(np.float64), X[:, 10:].astype(np.float64)
    l64, dP = oracle.cbce_backward(p, XV, XE, y)
    # autograd over the BF16 form: loss and gradient direction
    pt = torch.from_numpy(p).cuda().requires_grad_(True)
    f = nvgs.compact_mlp_function()
    z = f.apply(torch.from_numpy(X).cuda(), pt, ctx, "bf16")
    loss = torch.nn.functional.binary_cross_entropy_with_logits(z, torch.from_numpy(y).float().cuda())
    loss.backward()
    g = pt.grad.cpu().numpy().astype(np.float64)
    cos = float(np.dot(g, dP) / (np.linalg.norm(g) * np.linalg.norm(dP)))
    log(f"[cgrad] bf16: loss {loss.item():.6f} vs FP64 {l64:.6f}, gradient cosine {cos:.6f}")
    assert abs(loss.item() - l64) < 2e-3 * max(1.0, l64)
    assert cos >= 0.999
    # FP32 through autograd: the loss to FP32 accuracy
    pt32 = torch.from_numpy(p).cuda().requires_grad_(True)
    z32 = f.apply(torch.from_numpy(X).cuda(), pt32, ctx, "fp32")
    l32 = torch.nn.functional.binary_cross_entropy_with_logits(z32, torch.from_numpy(y).float().cuda())
    l32.backward()
    assert abs(l32.item() - l64) < 1e-5 * max(1.0, l64)
    assert _grad_close(pt32.grad.cpu().numpy().astype(np.float64), dP)[0] < 1e-4


def _compact_asset(n=2000, seed=6, d_min=1.0, d_max=8.0):
    return synth.make_compact(_small_asset(n=n, seed=seed), seed + 100, d_min=d_min, d_max=d_max)


@pytest.mark.parametrize("weighting", [0, 1])
def test_compact_training_step_matches_oracle(env, weighting):
    """One FP32 Adam step of the compact model on oracle labels: the GPU's
    batch loss equals the oracle's on the same SplitMix64-drawn pairs, and the
    first update agrees with the oracle's Adam step."""
    nvgs, ctx, torch = env
    a = _compact_asset()
    views = synth.label_views(4, seed=5, d_lo=2.0, d_hi=4.0, res=64)
    lab = oracle.labels(a, views)
    words = (a.n + 31) // 32
    packed = np.zeros((len(views), words * 32), np.uint8)
    packed[:, :a.n] = lab
    lab_words = np.packbits(packed, axis=1, bitorder="little").view(np.uint32).reshape(len(views), words)
    ctx.load_assets([a])
    p0 = a.mlp.params.astype(np.float32)
    pt = torch.from_numpy(p0.copy()).cuda()
    B, seed, lr = 1000, 91, 1e-3
    curve = ctx.train_visibility(0, views, pt, labels=torch.from_numpy(lab_words.view(np.int32)).cuda(), batch=B,
                                 steps=1, precision="fp32", lr=lr, seed=seed, weighting=weighting)
    g_idx, v_idx = oracle.sample_pairs(seed, 0, B, a.n, len(views))
    E, XE_all = oracle.cembed(a)
    XV = np.zeros((B, 10))
    for v in np.unique(v_idx):
        sel = np.flatnonzero(v_idx == v)
        XV[sel] = oracle.cinputs(a, synth.identity_instance(), views[v], g_idx[sel], E)[:, :10]
    XE = XE_all[g_idx]
    y = lab[v_idx, g_idx].astype(np.float64)
    w = None
    if weighting:  # each sample weighted by B / (2 n_class)
        npos = y.sum()
        w = np.where(y > 0.5, B / (2 * npos), B / (2 * (B - npos)))
    loss, dP = oracle.cbce_backward(p0, XV, XE, y, w=w)
    log(f"[ctrain] loss gpu {curve[0]:.6f} oracle {loss:.6f}")
    assert abs(curve[0] - loss) < 1e-5 * max(1.0, loss)
    p64 = p0.astype(np.float64)
    m = np.zeros_like(p64); v = np.zeros_like(p64)
    oracle.adam_step(p64, dP, m, v, 1, lr=lr)
    dg = pt.cpu().numpy().astype(np.float64) - p0
    do = p64 - p0
    big = np.abs(dP) > 1e-5 * np.abs(dP).max()
    agree = np.abs(dg - do) < 1e-6
    log(f"[ctrain] first update agrees on {agree[big].mean():.5f} of {big.sum()} parameters")
    assert agree[big].mean() > 0.995


def test_compact_training_reduces_loss(env):
    nvgs, ctx, torch = env
    a = _compact_asset(n=4000, seed=8, d_min=1.5, d_max=7.0)
    views = synth.label_views(24, seed=9, d_lo=2.0, d_hi=6.0, res=96)
    ctx.load_assets([a])
    pt = torch.from_numpy(a.mlp.params.astype(np.float32).copy()).cuda()
    curve = ctx.train_visibility(0, views, pt, batch=4096, steps=300, precision="bf16", lr=3e-3, seed=1)
    log(f"[ctrain] loss {curve[0]:.4f} -> {curve[-20:].mean():.4f}")
    assert np.all(np.isfinite(curve))
    assert curve[-20:].mean() < 0.8 * curve[:5].mean()
