"""Host-side logic of bench.py (CPU only): the per-stage work model and the
one-GPU contract."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _st(**kw):
    base = {"queried": 1000, "kept": 1000, "duplicates": 2000, "blend_tests": 10 ** 6}
    base.update(kw)
    return base


def test_projection_bytes_per_splat():
    # algorithmic: SH3 236 B Gaussian (56 B + 180 B of higher SH) read + 48 B splat written
    r = bench.stage_roof("project", 1.0, _st(kept=10 ** 6), 64, "fp32", 3, 32400)
    assert abs(r["achieved"] - 284e6 / 1e-3 / 1e9) < 1e-6
    # implementation: 48 B geometry + 48 floats of SH (192 B) read + 76 B written
    assert abs(r["impl_achieved"] - 316e6 / 1e-3 / 1e9) < 1e-6
    # SH0: 56 + 48 B; the implementation reads 3 floats rounded up to 4 (16 B)
    r0 = bench.stage_roof("project", 1.0, _st(kept=10 ** 6), 64, "fp32", 0, 32400)
    assert abs(r0["achieved"] - 104e6 / 1e-3 / 1e9) < 1e-6
    assert abs(r0["impl_achieved"] - 140e6 / 1e-3 / 1e9) < 1e-6


def test_sort_and_binning_bytes():
    st = _st(kept=10 ** 6, duplicates=3 * 10 ** 6)
    assert abs(bench.stage_roof("depth_sort", 1.0, st, 64, "fp32", 3, 1)["achieved"] - 64e6 / 1e-3 / 1e9) < 1e-6
    assert abs(bench.stage_roof("bin", 1.0, st, 64, "fp32", 3, 1)["achieved"] - 24e6 / 1e-3 / 1e9) < 1e-6
    assert abs(bench.stage_roof("tile_sort", 1.0, st, 64, "fp32", 3, 1)["achieved"] - 96e6 / 1e-3 / 1e9) < 1e-6
    # as built: four radix passes, the last also moving the rectangle and count (96 B per splat);
    # binning: the count scan and the emitter (28 B per splat) + 8 B per entry
    assert abs(bench.stage_roof("depth_sort", 1.0, st, 64, "fp32", 3, 1)["impl_achieved"] - 96e6 / 1e-3 / 1e9) < 1e-6
    assert abs(bench.stage_roof("bin", 1.0, st, 64, "fp32", 3, 1)["impl_achieved"] - 52e6 / 1e-3 / 1e9) < 1e-6


@pytest.mark.parametrize("keys,passes", [(255, 1), (256, 1), (257, 2), (32400, 2), (65536, 2), (65537, 3),
                                         (259200, 3)])
def test_tile_sort_passes_follow_the_key_width(keys, passes):
    r = bench.stage_roof("tile_sort", 1.0, _st(duplicates=10 ** 6), 64, "fp32", 3, keys)
    assert abs(r["impl_achieved"] - (20 * passes + 4) * 1e6 / 1e-3 / 1e9) < 1e-6


def test_traffic_is_keyed_by_workload():
    # counters taken on one workload are never reported for another
    assert bench.measured_traffic("project", "batched8x1080p") is None
    assert bench.measured_traffic("project", "no such workload") is None


def test_mlp_flop_model():
    r = bench.stage_roof("cull_mlp", 2.0, _st(queried=10 ** 6), 64, "fp32", 3, 1)
    assert abs(r["achieved"] - 16512e6 / 2e-3 / 1e12) < 1e-9
    assert bench.FLOP_PER_QUERY[32] == 2 * (4 * 32 + 32 * 32 + 32)
    assert r["peak"] == 157.3 and r["bound"] == "mfma"


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
