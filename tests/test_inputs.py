"""Checks of the synthetic input recipes (CPU only): surface-aligned
Gaussians, the training-view offset rule and the view samplings."""
import math

import numpy as np

import synth


def _third_axis(q):
    w, x, y, z = q.astype(np.float64)
    return np.stack([2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y)])


def test_surface_frames_put_the_third_axis_on_the_normal():
    g = np.random.default_rng(3)
    nrm = g.standard_normal((3, 500))
    nrm /= np.linalg.norm(nrm, axis=0)
    nrm[:, :3] = [[0, 0, 0], [0, 0, 0], [1, -1, 1]]  # both poles exactly (the antipode needs the half turn)
    q = synth.surface_frames(nrm, np.random.default_rng(4))
    np.testing.assert_allclose(np.linalg.norm(q.astype(np.float64), axis=0), 1.0, atol=1e-6)
    np.testing.assert_allclose(_third_axis(q), nrm, atol=1e-6)
    # the twist is random: the first axes of equal normals differ
    q2 = synth.surface_frames(np.repeat(nrm[:, 3:4], 50, axis=1), np.random.default_rng(5)).astype(np.float64)
    w, x, y, z = q2
    first = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)])
    assert np.std(first, axis=1).max() > 0.3


def test_aligned_assets_lie_flat_on_their_surface():
    for shape in ("torus", "sphere", "box", "helix"):
        a = synth.make_asset(shape, 2000, 0, 11, aligned=True)
        b = synth.make_asset(shape, 2000, 0, 11)
        np.testing.assert_array_equal(a.mean, b.mean)          # positions and the other draws unchanged
        np.testing.assert_array_equal(a.opacity, b.opacity)
        np.testing.assert_array_equal(a.scale[:2], b.scale[:2])
        np.testing.assert_allclose(a.scale[2], b.scale[2] * np.float32(0.1), rtol=1e-6)
        _, nrm = synth.SHAPES[shape](2000, synth.rng(11), normals=True)
        np.testing.assert_allclose(_third_axis(a.quat), nrm, atol=1e-5)
    # sphere: the normal is the radial direction (up to the jitter)
    s = synth.make_asset("sphere", 2000, 0, 12, aligned=True)
    radial = s.mean / np.linalg.norm(s.mean, axis=0)
    assert np.min(np.sum(radial * _third_axis(s.quat), axis=0)) > 0.99


def test_view_offset_rule_keeps_the_asset_in_the_frame():
    """Offset zero at the near distance, at most r * d_max / d_min at the far
    one, growing linearly; with Eq. 1's range the asset stays in the image."""
    for shape in ("torus", "helix"):
        r = synth.SHAPE_HALF_DIAG[shape]
        d_lo, d_hi = synth.eq1_range(shape)
        views = synth.label_views(400, seed=9, d_lo=d_lo, d_hi=d_hi, res=64, offset=1.0, radius=r)
        t = math.tan(math.radians(50.0) / 2)
        for cam in views:
            pos = cam.pos.astype(np.float64)
            d = np.linalg.norm(pos)
            lam = (d - d_lo) / (d_hi - d_lo)
            # the asset centre's offset from the view axis, in units of the half frame at its depth
            c_cam = cam.R.astype(np.float64) @ (-pos)
            frac = math.hypot(c_cam[0], c_cam[1]) / (c_cam[2] * t)
            assert frac <= r * (d_hi / d_lo) * lam / (c_cam[2] * t) + 1e-4
            assert frac + r / (c_cam[2] * t) <= 1.0 + 0.05  # whole bounding sphere within the frame (5 % slack)
        # the bound shrinks to zero at the minimum distance: views within 1 % of it look almost at the centre
        close = [c for c in views if np.linalg.norm(c.pos.astype(np.float64)) < d_lo + 0.01 * (d_hi - d_lo)]
        assert close
        for cam in close:
            c_cam = cam.R.astype(np.float64) @ (-cam.pos.astype(np.float64))
            assert math.hypot(c_cam[0], c_cam[1]) < 0.01 * r * d_hi / d_lo + 1e-4


def test_longlat_and_fibonacci_directions():
    d = synth.longlat_sphere(2000)
    assert d.shape == (2000, 3)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    lat = np.arcsin(d[:, 2])
    # equal angular steps: the rings crowd towards the poles compared with the area-uniform Fibonacci spiral
    f = synth.fibonacci_sphere(2000)
    assert np.mean(np.abs(lat) > math.radians(60)) > 1.5 * np.mean(np.abs(np.arcsin(f[:, 2])) > math.radians(60))
