"""Differentiation form: the hand-written MLP backward, the autograd
function, renderer-made labels and training, against the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

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


def _batch(B, seed):
    g = np.random.default_rng(seed)
    p = synth.mlp_params(64, synth.rng(seed)).astype(np.float32)
    X = g.uniform(-1, 1, (B, 72)).astype(np.float32)
    y = (g.uniform(0, 1, B) > 0.5).astype(np.float64)
    return p, X, y


def _grad_close(dg, do, tol=1e-3):
    floor = 1e-6 * np.max(np.abs(do))
    rel = np.abs(dg - do) / np.maximum(np.abs(do), floor)
    return np.linalg.norm(dg - do) / np.linalg.norm(do), rel


@pytest.mark.parametrize("B", [300, 1024, 65536])  # 65,536: the differentiation workload's batch
def test_mlp_forward_backward_fp32_vs_oracle(env, B):
    nvgs, ctx, torch = env
    p, X, y = _batch(B, 5 + B)
    z64, scale = oracle.mlp_forward(p, 64, X)
    zg = ctx.mlp_forward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    assert np.all(np.abs(zg - z64) <= 1e-5 * np.maximum(np.abs(z64), scale))
    dlog = ((1 / (1 + np.exp(-z64)) - y) / B).astype(np.float32)
    loss, dP, dX = oracle.bce_backward(p, 64, X, y, want_dx=True)
    dp_g, dx_g = ctx.mlp_backward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(), torch.from_numpy(dlog).cuda())
    nrm, rel = _grad_close(dp_g.cpu().numpy().astype(np.float64), dP)
    log(f"[grad] B={B}: param grad rel norm err {nrm:.2e}, max rel {rel.max():.2e}")
    assert nrm < 1e-3 and np.mean(rel < 1e-3) > 0.999
    nrm_x, rel_x = _grad_close(dx_g.cpu().numpy().astype(np.float64), dX)
    assert nrm_x < 1e-3


def test_mlp_backward_bf16_cosine(env):
    nvgs, ctx, torch = env
    B = 2048
    p, X, y = _batch(B, 9)
    z64, _ = oracle.mlp_forward(p, 64, X)
    dlog = ((1 / (1 + np.exp(-z64)) - y) / B).astype(np.float32)
    _, dP = oracle.bce_backward(p, 64, X, y)
    dp_g, _ = ctx.mlp_backward(torch.from_numpy(p).cuda(), torch.from_numpy(X).cuda(), torch.from_numpy(dlog).cuda(),
                               precision="bf16", want_dx=False)
    g = dp_g.cpu().numpy().astype(np.float64)
    cos = float(np.dot(g, dP) / (np.linalg.norm(g) * np.linalg.norm(dP)))
    log(f"[grad] bf16 cosine similarity to FP64 gradient {cos:.6f}")
    assert cos >= 0.999


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


def _small_asset(n=3000, seed=4):
    a = synth.make_asset("torus", n, 0, seed, width=64, cam_scale=1.0 / 20.0, d_max=20.0)
    a.opacity[:] = np.clip(a.opacity * 1.2, 0, 1)
    a.scale[:] *= 2.0
    return a


@pytest.mark.parametrize("aux", [0, 6])
def test_labels_match_oracle(env, aux):
    """Labels rendered by the library equal the oracle's (largest alpha*T over
    the view and its auxiliary views above 1/255) away from the threshold."""
    nvgs, ctx, torch = env
    a = _small_asset()
    views = synth.label_views(6, seed=3, d_lo=2.0, d_hi=4.0, res=96, offset=0.2)
    ang = math.radians(5.0)
    ctx.load_assets([a])
    lab = ctx.make_labels(0, views, aux=aux, aux_angle=ang).cpu().numpy().view(np.uint32)
    bits = np.unpackbits(lab.view(np.uint8).reshape(len(views), -1), axis=1, bitorder="little")[:, :a.n]
    cb = np.stack([oracle.contributions(a, [v] + oracle.aux_views(v, aux, ang)).max(axis=0) for v in views])
    ref = cb > 1 / 255
    diff = bits.astype(bool) != ref
    near = np.abs(cb - 1 / 255) < 2e-3 / 255
    log(f"[labels aux={aux}] {ref.mean():.3f} visible; mismatches {diff.sum()} (near threshold {np.sum(diff & near)})")
    assert 0.1 < ref.mean() < 0.95
    assert np.sum(diff & ~near) <= max(2, 1e-4 * diff.size)


def test_labels_full_size(env):
    """Labels of the differentiation workload's own asset (500k SH3
    Gaussians) on three of its 512 label views at 512x512, against the
    oracle's largest alpha*T per Gaussian, away from the threshold."""
    nvgs, ctx, torch = env
    sc = synth.scene_train()
    a = sc.assets[0]
    views = synth.label_views(512, seed=synth.SEED_BASE + 5, d_lo=1.5, d_hi=20.0, res=512)
    views = [views[j] for j in (0, 171, 342)]
    ctx.load_assets([a])
    lab = ctx.make_labels(0, views).cpu().numpy().view(np.uint32)
    bits = np.unpackbits(lab.view(np.uint8).reshape(len(views), -1), axis=1, bitorder="little")[:, :a.n]
    cb = oracle.contributions(a, views)
    ref = cb > 1 / 255
    diff = bits.astype(bool) != ref
    near = np.abs(cb - 1 / 255) < 2e-3 / 255
    log(f"[labels full size] {a.n} Gaussians x {len(views)} views: {ref.mean():.3f} visible; mismatches "
        f"{diff.sum()} (near threshold {np.sum(diff & near)})")
    assert 0.01 < ref.mean() < 0.95
    assert np.sum(diff & ~near) <= max(2, 1e-4 * diff.size)


@pytest.mark.parametrize("weighting", [0, 1])
def test_training_step_matches_oracle(env, weighting):
    """One FP32 Adam step on oracle labels: the GPU's batch loss equals the
    oracle's on the same SplitMix64-drawn pairs, and the first Adam update
    (lr * sign(g) where |g| >> eps) agrees."""
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
    loss, dP = oracle.bce_backward(p0, 64, X, y, w=w)
    log(f"[train] loss gpu {curve[0]:.6f} oracle {loss:.6f}")
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


def test_training_reduces_loss(env):
    nvgs, ctx, torch = env
    a = _small_asset(n=4000, seed=8)
    views = synth.label_views(24, seed=9, d_lo=2.0, d_hi=6.0, res=96)
    ctx.load_assets([a])
    pt = torch.from_numpy(a.mlp.params.astype(np.float32).copy()).cuda()
    curve = ctx.train_visibility(0, views, pt, batch=4096, steps=300, precision="bf16", lr=3e-3, seed=1)
    log(f"[train] loss {curve[0]:.4f} -> {curve[-20:].mean():.4f}")
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
