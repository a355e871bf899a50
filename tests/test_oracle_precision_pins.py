"""Pins of the oracle's reduced-precision checker, footprint and learning-rate
schedule against things other than itself: the OCP E4M3 definition and
PyTorch's float8 / bfloat16 casts (library routines), hand-derived scale
values, an independent NumPy emulation of the precision form, brute force
over pixel columns, and closed forms of the schedule.  CPU only."""
import math

import numpy as np
import pytest
import torch

import synth
from synth import Camera, Scene

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# ---------------------------------------------------------------------------
# OCP FP8 E4M3 (the precision form's 8-bit operands)
# ---------------------------------------------------------------------------
def e4m3_from_definition(code: int) -> float:
    """Value of an E4M3 code from the OCP 8-bit floating point definition:
    sign, 4 exponent bits with bias 7, 3 mantissa bits; exponent 0 is
    subnormal (2^-6 * m/8); exponent 15 with mantissa 7 is NaN; no infinity."""
    s = -1.0 if code & 0x80 else 1.0
    e, m = (code >> 3) & 0xF, code & 0x7
    if e == 15 and m == 7:
        return float("nan")
    if e == 0:
        return s * 2.0 ** -6 * (m / 8.0)
    return s * 2.0 ** (e - 7) * (1.0 + m / 8.0)


def test_e4m3_codes_definition_matches_torch():
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    via_torch = codes.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    mine = np.array([e4m3_from_definition(c) for c in range(256)])
    assert np.array_equal(np.isnan(mine), np.isnan(via_torch))
    ok = ~np.isnan(mine)
    assert np.array_equal(mine[ok], via_torch[ok])
    assert np.nanmax(mine) == 448.0 and np.nanmin(mine[mine > 0]) == 2.0 ** -9


def _positive_e4m3():
    vals = sorted({e4m3_from_definition(c) for c in range(0x7F)})  # 0 .. 448
    assert len(vals) == 127 and vals[0] == 0.0 and vals[-1] == 448.0
    return vals


def test_oracle_e4m3_round_trips_every_finite_code(orc):
    for c in range(256):
        v = e4m3_from_definition(c)
        if math.isnan(v):
            continue
        assert orc.to_e4m3(v) == v, (c, v)


def test_oracle_e4m3_ties_to_even_and_neighbours_match_torch(orc):
    vals = _positive_e4m3()
    xs = []
    for i in range(len(vals) - 1):
        lo, hi = vals[i], vals[i + 1]
        mid = np.float32(0.5 * (lo + hi))  # exact in float32 (5 significant bits)
        assert float(mid) == 0.5 * (lo + hi)
        below = np.nextafter(mid, np.float32(0))
        above = np.nextafter(mid, np.float32(np.inf))
        # the tie goes to the code with an even mantissa (the even code)
        lo_code = i  # positive codes are ordered like their values
        even = lo if lo_code % 2 == 0 else hi
        assert orc.to_e4m3(float(mid)) == even, (lo, hi)
        assert orc.to_e4m3(float(below)) == lo
        assert orc.to_e4m3(float(above)) == hi
        xs += [mid, below, above, np.float32(lo + 0.3 * (hi - lo)), np.float32(lo + 0.7 * (hi - lo))]
    x = np.array(xs, np.float32)
    x = np.concatenate([x, -x])
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = orc.to_e4m3(x.astype(np.float64))
    assert np.array_equal(got, ref)


def test_oracle_e4m3_saturates_at_448(orc):
    # below the midpoint to the next binade's first step (464) the nearest value is 448;
    # beyond it the precision form saturates (reading of the format: no infinity, clamp)
    for v in [448.0, 450.0, 463.9, 464.0, 479.0, 480.0, 1e4, 3e38]:
        assert orc.to_e4m3(v) == 448.0 and orc.to_e4m3(-v) == -448.0
    ref = torch.tensor([450.0, 463.9], dtype=torch.float32).to(torch.float8_e4m3fn).to(torch.float64)
    assert ref.tolist() == [448.0, 448.0]


def test_oracle_e4m3_subnormal_spacing(orc):
    q = 2.0 ** -9
    for k in range(8):
        assert orc.to_e4m3(k * q) == k * q
        assert orc.to_e4m3(k * q + 0.49 * q) == k * q
    assert orc.to_e4m3(0.5 * q) == 0.0        # tie between 0 (even) and 2^-9 (odd)
    assert orc.to_e4m3(1.5 * q) == 2 * q      # tie between 1 (odd) and 2 (even)
    assert orc.to_e4m3(2.0 ** -6 - 0.5 * q) == 2.0 ** -6  # tie 7q | 8q: 8q = 2^-6 has mantissa 0


# ---------------------------------------------------------------------------
# BF16
# ---------------------------------------------------------------------------
def test_oracle_bf16_matches_torch_and_bit_level_ties(orc):
    rng = np.random.default_rng(7)
    x = (rng.standard_normal(20000) * np.exp2(rng.integers(-60, 60, 20000))).astype(np.float32)
    # exact ties: the 16 dropped bits are 0x8000
    u = rng.integers(0, 2 ** 31, 4000, dtype=np.uint64).astype(np.uint32)
    ties = ((u & np.uint32(0x7F7F0000)) | np.uint32(0x8000)).view(np.float32)
    x = np.concatenate([x, ties, -ties, np.float32([0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 3.3895e38])])
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = orc.to_bf16(x.astype(np.float64))
    ok = np.isfinite(ref)
    assert np.array_equal(got[ok], ref[ok])
    # hand cases: 1 + 2^-8 sits halfway between 1 (even) and 1 + 2^-7 (odd) -> 1;
    # 1 + 3 2^-8 halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even) -> 1 + 2^-6
    assert orc.to_bf16(1.0 + 2 ** -8) == 1.0
    assert orc.to_bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


# ---------------------------------------------------------------------------
# FP8 per-layer scales: hand-derived values
# ---------------------------------------------------------------------------
def _unpack(P, W):
    o = 0
    W1 = P[o:o + W * 72].reshape(W, 72); o += W * 72
    b1 = P[o:o + W]; o += W
    W2 = P[o:o + W * W].reshape(W, W); o += W * W
    b2 = P[o:o + W]; o += W
    W3 = P[o:o + W * W].reshape(W, W); o += W * W
    b3 = P[o:o + W]; o += W
    wo = P[o:o + W]; o += W
    bo = P[o]
    return W1, b1, W2, b2, W3, b3, wo, bo


def test_fp8_scales_on_a_hand_built_net(orc):
    W = 64
    P = np.zeros(72 * W + W + 2 * (W * W + W) + W + 1)
    W1, b1, W2, b2, W3, b3, wo, bo = _unpack(P, W)  # views into P
    W1[5, 3] = 0.7      # the largest weight of layer 1's Gaussian half
    W1[10, 50] = -3.0   # camera half: not an MFMA operand, but in the row-sum bound
    b1[10] = 1.0        # row 10: |W1| sum + |b1| = 4  -> bound on |h1| is 4
    W2[0, :] = 0.25     # row 0 sums to 16 -> bound on |h2| is 16 * 4 + |b2[0]|
    b2[0] = 0.5
    W3[1, 2] = -5.0
    sc = orc.fp8_scales(P, W)
    # largest powers of two with scale * max <= 448:
    # 448 / 0.7 = 640 -> 512; 448 / 0.25 = 1792 -> 1024; 448 / 5 = 89.6 -> 64;
    # inputs |gamma| <= 1: 448 -> 256; |h1| <= 4: 112 -> 64; |h2| <= 64.5: 6.95 -> 4
    sw1, sw2, sw3, sag, sa1, sa2 = 512.0, 1024.0, 64.0, 256.0, 64.0, 4.0
    want = [1 / (sw1 * sag), 1 / (sw2 * sa1), 1 / (sw3 * sa2), sa1, sa2, sag, sw1, sw2, sw3]
    assert list(sc) == want


def test_fp8_scales_bound_the_activations_and_are_maximal(orc):
    W = 64
    P = synth.mlp_params(W, synth.rng(3)).astype(np.float64)
    W1, b1, W2, b2, W3, b3, wo, bo = _unpack(P, W)
    sc = orc.fp8_scales(P, W)
    sa1, sa2, sag, sw1, sw2, sw3 = sc[3], sc[4], sc[5], sc[6], sc[7], sc[8]
    for s in (sa1, sa2, sag, sw1, sw2, sw3):
        assert s > 0 and math.frexp(s)[0] == 0.5  # a power of two
    # the weight scales are the largest powers of two that keep every operand <= 448
    for s, m in ((sw1, np.abs(W1[:, :36]).max()), (sw2, np.abs(W2).max()), (sw3, np.abs(W3).max())):
        assert s * m <= 448 < 2 * s * m
    # activations of any input with |gamma| <= 1 stay within 448 after scaling
    g = np.random.default_rng(5).uniform(-1, 1, (20000, 72))
    g[:4] = np.sign(W1[np.argmax(np.abs(W1).sum(1))])  # the worst case of the row-sum bound
    h1 = np.maximum(g @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    assert np.abs(h1).max() * sa1 <= 448 and np.abs(h2).max() * sa2 <= 448
    # the layer-1 bound is attained by the sign pattern above, so its scale is maximal
    assert 2 * sa1 * np.abs(h1).max() > 448


# ---------------------------------------------------------------------------
# the reduced-precision forward against an independent NumPy emulation
# ---------------------------------------------------------------------------
def _round_lib(x, prec):
    t = torch.from_numpy(np.asarray(x, np.float64).astype(np.float32))
    dt = torch.bfloat16 if prec == "bf16" else torch.float8_e4m3fn
    return t.to(dt).to(torch.float64).numpy()


def _f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def emulate_precision_form(P, W, X, prec, scales):
    """The precision form as stated for the kernels: every operand the per-query
    GEMM chain consumes on MFMA (the Gaussian features and W1's Gaussian half,
    h1 and W2, h2 and W3) is rounded to BF16 / E4M3 after its power-of-two
    scale, products are exact and accumulate to one FP32 value per output;
    the per-(camera, instance) camera half of layer 1 (with b1), the biases,
    ReLU and the output layer are FP32 values."""
    W1, b1, W2, b2, W3, b3, wo, bo = _unpack(np.asarray(P, np.float64), W)
    if prec == "fp8":
        invU, inv2, inv3, sa1, sa2, sag, sw1, sw2, sw3 = scales
    else:
        invU = inv2 = inv3 = sa1 = sa2 = sag = sw1 = sw2 = sw3 = 1.0
    q = lambda v: _round_lib(v, prec)  # noqa: E731
    g = q(_f32(X[:, :36]) * sag)
    U = g @ q(W1[:, :36] * sw1).T                                   # exact products, FP64 sum
    cam = _f32(X[:, 36:] @ W1[:, 36:].T + b1)                       # FP32 camera half + b1
    h1 = q(_f32(np.maximum(_f32(_f32(U) * invU + cam), 0)) * sa1)
    a2 = h1 @ q(W2 * sw2).T
    h2 = q(_f32(np.maximum(_f32(a2) * inv2 + b2, 0)) * sa2)
    a3 = h2 @ q(W3 * sw3).T
    h3 = np.maximum(_f32(a3) * inv3 + b3, 0)
    return h3 @ wo + bo, np.abs(h3) @ np.abs(wo) + abs(bo)


@pytest.mark.parametrize("W", [64, 128])
@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_forward_q_matches_independent_emulation(orc, W, prec):
    P = synth.mlp_params(W, synth.rng(11 + W)).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(W)
    ang = rng.uniform(-4, 4, (3000, 6))
    X = np.concatenate([np.sin(ang[:, :3, None] * 2.0 ** np.arange(6)), np.cos(ang[:, :3, None] * 2.0 ** np.arange(6)),
                        np.sin(ang[:, 3:, None] * 2.0 ** np.arange(6)), np.cos(ang[:, 3:, None] * 2.0 ** np.arange(6))],
                       axis=2).reshape(3000, 72)  # encoded-like inputs in [-1, 1]
    sc = orc.fp8_scales(P, W)
    want, scale = emulate_precision_form(P, W, X, prec, sc)
    got = orc.mlp_forward_q(P, W, X, prec)
    err = np.abs(got - want) / scale
    # equal up to FP64 summation order (an FP32 rounding boundary hit by ~1e-16 is
    # the only way they could differ, at most a handful of values)
    assert np.mean(err < 1e-9) > 0.999 and np.max(err) < 1e-2
    # and the rounding is not a no-op: the FP64 MLP differs visibly
    z64, _ = orc.mlp_forward(P, W, X)
    assert np.median(np.abs(z64 - want) / scale) > (1e-5 if prec == "bf16" else 1e-4)


# ---------------------------------------------------------------------------
# footprint: exact (not merely conservative) against brute force over columns
# ---------------------------------------------------------------------------
def _axis_cam(W, H):
    return Camera(pos=np.zeros(3, np.float32), R=np.eye(3, dtype=np.float32), fovy=math.radians(60.0),
                  width=W, height=H, near=0.2)


def _one(mean, scale, o):
    return synth.Asset(mean=np.asarray(mean, np.float32).reshape(3, 1),
                       scale=np.asarray(scale, np.float32).reshape(3, 1),
                       quat=np.asarray((1, 0, 0, 0), np.float32).reshape(4, 1),
                       opacity=np.asarray([o], np.float32), sh=np.zeros((3, 1), np.float32), sh_degree=0,
                       mlp=synth.MLPSpec(params=synth.mlp_params(8, synth.rng(0)), width=8))


@pytest.mark.parametrize("axis", [0, 1])
def test_footprint_is_the_exact_alpha_box(orc, axis):
    """Gaussians on the camera's x = 0 or y = 0 plane with identity rotation
    project to axis-aligned ellipses (Sigma2D off-diagonal 0), whose extent
    along the other axis is reached on the row (column) through the centre.
    There alpha = o exp(-d^2 / (2 Sigma2D_ii)), so the columns (rows) a splat
    must cover are found by brute force from the alpha definition; the
    rectangle must hold all of them and at most one more on each side, and
    such an extra line only within the FP32 safety margin (alpha within 1 %
    of 1/255)."""
    W, H = 220, 200
    cam = _axis_cam(W, H)
    rng = np.random.default_rng(40 + axis)
    extra = 0
    for k in range(300):
        z = rng.uniform(1.0, 12.0)
        off = rng.uniform(-0.4, 0.4) * z
        mean = (off, 0.0, z) if axis == 0 else (0.0, off, z)
        scale = np.exp(rng.uniform(-5.0, -1.0, 3))
        o = rng.uniform(0.01, 1.0)
        sc = Scene(assets=[_one(mean, scale, o)], instances=[synth.identity_instance(0)], cameras=[cam])
        rec, prect = orc.project(sc, cam, np.zeros(1, np.int64))
        r, pr = rec[0], prect[0]
        assert abs(r[3]) < 1e-15  # axis-aligned
        c0, s_ii, lo, hi, n = (r[0], r[2], pr[0], pr[1], W) if axis == 0 else (r[1], r[4], pr[2], pr[3], H)
        d = np.arange(n) + 0.5 - c0
        alpha = o * np.exp(-d * d / (2.0 * s_ii))  # the 0.99 clamp does not affect alpha >= 1/255
        need = np.flatnonzero(alpha >= 1.0 / 255.0)
        if len(need) == 0:
            assert lo > hi or all(alpha[lo:hi + 1] >= 0.99 / 255.0)
            continue
        assert lo <= need.min() and need.max() <= hi
        assert need.min() - lo <= 1 and hi - need.max() <= 1
        for line in range(lo, hi + 1):
            if line < need.min() or line > need.max():
                extra += 1
                assert alpha[line] >= 0.99 / 255.0, (k, line, alpha[line] * 255)
    assert extra < 30  # the margin rarely adds a line


# ---------------------------------------------------------------------------
# learning-rate schedule of Sec. 4.1: closed-form values
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("T", [1, 2, 5, 10, 37, 5000])
def test_lr_schedule_closed_forms(orc, T):
    lr, lf = 2e-3, 2e-4
    s = np.array([orc.lr_schedule(lr, lf, T, t) for t in range(T)])
    Tw = max(1, int(round(0.2 * T)))
    assert np.all(s > 0)
    # cosine warm-up: reaches lr at the last warm-up step, rises monotonically,
    # and is at half of lr halfway (when the warm-up has an even length)
    assert s[Tw - 1] == pytest.approx(lr, rel=1e-15)
    assert np.all(np.diff(s[:Tw]) > 0)
    if Tw % 2 == 0:
        assert s[Tw // 2 - 1] == pytest.approx(lr / 2, rel=1e-14)
    if T > Tw:
        # exponential decay: starts at lr, ends at lr_final, constant ratio per step
        assert s[-1] == pytest.approx(lf, rel=1e-14)
        if T - Tw > 1:
            assert s[Tw] == pytest.approx(lr, rel=1e-15)
            r = s[Tw + 1:] / s[Tw:-1]
            assert np.allclose(r, (lf / lr) ** (1.0 / (T - 1 - Tw)), rtol=1e-12)
    if T == 5000:
        assert Tw == 1000 and s[499] == pytest.approx(1e-3, rel=1e-14)
        assert s[1000 + 1333] == pytest.approx(2e-3 * 0.1 ** (1333 / 3999), rel=1e-12)
