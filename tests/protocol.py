"""Decision-margin protocol shared by the GPU parity tests.

FP32 kernels and the FP64 oracle can disagree only where a discrete decision
(frustum or keep test, alpha >= 1/255, the 1e-4 stop, the depth order of two
fragments, a footprint bound crossing a pixel line) is closer to its threshold
than FP32 resolves.  The oracle reports each item's FP64 margin; an item that
differs is excused only when that margin is below the bound stated here, and
every excusal is counted and logged.  Pixels must be within 1e-4 absolute
unless a decision on that pixel was within margin.
"""
import sys

import numpy as np

# frustum / keep decisions: relative FP64 margin below which FP32 may differ
MARGIN = 1e-5
# alpha and stop decisions at a pixel (relative margin of alpha to 1/255 and
# of the new transmittance to 1e-4).  The kernel's alpha carries a relative
# error of about |log2 alpha| * 2^-23 from the base-2 exponential and the
# FP32 quadratic form (its centre is tile-relative and held to ~48 bits), and
# the transmittance compounds alpha's error by alpha / (1 - alpha) per blended
# fragment (up to 99x at the 0.99 clamp) over the fragments before the stop,
# so stop decisions need the wider bound.
MARGIN_ALPHA = 1e-4
# depth order: FP32 depth keys resolve ~6e-8 relative; two fragments whose
# FP64 depths are closer than this may be blended in either order
MARGIN_DEPTH = 1e-6
# footprint bounds: a bound position u -/+ e - 0.5 -/+ w within this many
# pixels of an integer may round either way in FP32 (half an ulp of the
# centre below 2048 px is 6.1e-5 px; the extent's FP32 relative error is a
# few 1e-7, and three roundings of the sum)
RECT_MARGIN_PX = 2.5e-4
RECT_MARGIN_REL = 2e-6


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_pixels(img, ref, label, tol=1e-4):
    """Pixels of one camera against the oracle's render: every pixel whose
    decisions all had margins above the bounds is within `tol`.  Logs the
    excused pixels by the margin that excused them.  Returns the largest error
    of the pixels that were not excused."""
    dimg = np.abs(np.asarray(img, np.float64) - ref["image"]).max(axis=2)
    bad = dimg > tol
    ma, md = ref["margin"][..., 0], ref["margin"][..., 1]
    tie_a = ma < MARGIN_ALPHA
    tie_d = md < MARGIN_DEPTH
    excused = bad & (tie_a | tie_d)
    other = float(np.max(np.where(excused, 0.0, dimg))) if dimg.size else 0.0
    bins = [0.0, 1e-7, 1e-6, 1e-5, 1e-4, np.inf]
    hist = np.histogram(ma[bad & tie_a & ~tie_d], bins=bins)[0] if bad.any() else np.zeros(len(bins) - 1, int)
    log(f"[pixels] {label}: max err {dimg.max():.3e}; {int(bad.sum())} of {dimg.size} above {tol:g}, "
        f"excused {int(excused.sum())} (depth order {int(np.sum(bad & tie_d))}, alpha/stop margins "
        f"<1e-7 {hist[0]}, <1e-6 {hist[1]}, <1e-5 {hist[2]}, <1e-4 {hist[3]}); the others within {other:.2e}")
    unexcused = bad & ~excused
    if unexcused.any():
        ys, xs = np.nonzero(unexcused)
        for y, x in list(zip(ys, xs))[:8]:
            log(f"[pixels]   unexcused ({x}, {y}): err {dimg[y, x]:.3e}, alpha/stop margin {ma[y, x]:.3e}, "
                f"depth margin {md[y, x]:.3e}")
    assert not unexcused.any(), f"{label}: {int(unexcused.sum())} pixels beyond {tol:g} with no decision in margin"
    return other


def rect_bound_margin(rec, W, H):
    """Distance in pixels of each FP64 footprint bound position from the pixel
    line where it would round differently, per splat (inf for bounds clamped
    to the image border), and whether that distance is within the FP32 margin
    of the kernel's centre and extent.  rec: oracle records (u 0, v 1,
    opacity 9, ex 13, ey 14)."""
    u, v, ex, ey = rec[:, 0], rec[:, 1], rec[:, 13], rec[:, 14]
    wx, wy = 1e-4 * ex + 1e-3, 1e-4 * ey + 1e-3
    pos = np.stack([u - ex - 0.5 - wx, u + ex - 0.5 + wx, v - ey - 0.5 - wy, v + ey - 0.5 + wy], axis=1)
    d = np.abs(pos - np.round(pos))
    # a bound beyond the image edge is clamped: its rounding cannot matter
    d[:, 0] = np.where(pos[:, 0] <= -1.0, np.inf, d[:, 0])
    d[:, 1] = np.where(pos[:, 1] >= W, np.inf, d[:, 1])
    d[:, 2] = np.where(pos[:, 2] <= -1.0, np.inf, d[:, 2])
    d[:, 3] = np.where(pos[:, 3] >= H, np.inf, d[:, 3])
    ext = np.stack([ex, ex, ey, ey], axis=1)
    within = d < RECT_MARGIN_PX + RECT_MARGIN_REL * ext
    # the empty-footprint test 255 o >= 1 on the same FP32 opacity
    o_close = np.abs(255.0 * rec[:, 9] - 1.0) < 1e-6
    return d.min(axis=1), within.any(axis=1) | o_close
