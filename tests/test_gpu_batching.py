"""Batching form: several cameras in one frame, the persistent (captured HIP
graph) frame, capacities and overflow, MLP block shapes and the autotuner,
all through the C ABI and against the FP64 oracle or the eager frame."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import scenes
from tests.protocol import check_pixels

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
    sc = scenes.batched_small()
    return nvgs, torch, sc


_SCENES = {}


def scene_of(kind):
    """The batching scene with the frequency-encoded MLP, or with the compact form."""
    if kind not in _SCENES:
        _SCENES[kind] = scenes.batched_small() if kind == "frequency" else scenes.batched_compact()
    return _SCENES[kind]


def make_ctx(nvgs, sc):
    ctx = nvgs.Context(0)
    ctx.load_assets(sc.assets)
    ctx.set_instances(sc.instances)
    return ctx


def ring(sc, frame):
    """Cameras of the ring turned by `frame` degrees (same assets and instances)."""
    c = sc.cameras[0]
    return synth.ring_cameras(len(sc.cameras), frame, 8.0, 2.5, (c.width, c.height))


@pytest.mark.parametrize("kind", ["frequency", "compact"])
def test_multi_camera_frame_matches_oracle(env, kind):
    nvgs, torch, _ = env
    sc = scene_of(kind)
    log(f"[multi] MLP {kind}")
    ctx = make_ctx(nvgs, sc)
    C = len(sc.cameras)
    img, stats = ctx.render(sc.cameras, tile=16, keep_debug=True, stats=True)
    dbg = ctx.debug_buffers()
    st, _ = ctx.query_visibility(sc.cameras)
    img, st = img.cpu().numpy().astype(np.float64), st.cpu().numpy()
    pair = dbg["pair"].cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    ctx.close()
    P = st.shape[1]
    log(f"[multi] {C} cameras, {P} pairs each, {stats['kept']} splats, {stats['duplicates']} entries")
    # compaction over the (camera, instance, Gaussian) order
    kept = [np.flatnonzero(st[k] == 2) for k in range(C)]
    assert np.array_equal(pair, np.concatenate([k * P + kept[k] for k in range(C)]))
    assert all(len(x) > 0 for x in kept)
    # tile keys: camera-major, ascending, each entry's camera is its splat's
    sk = dbg["sorted_key"].cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    sid = dbg["sorted_id"].cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    n_tiles = dbg["tiles_x"] * dbg["tiles_y"]
    assert np.all(np.diff(sk) >= 0)
    cam_of_splat = np.repeat(np.arange(C), [len(x) for x in kept])
    assert np.array_equal(sk // n_tiles, cam_of_splat[sid])
    # pixels of every camera vs the FP64 oracle on the same kept pairs
    for k, cam in enumerate(sc.cameras):
        rec, prect = oracle.project(sc, cam, kept[k])
        ref = oracle.render_camera(rec, prect, cam, 16, sc.bg)
        log(f"[multi] camera {k}: {len(kept[k])} splats")
        check_pixels(img[k], ref, f"multi-camera {kind} camera {k}")


@pytest.mark.parametrize("kind", ["frequency", "compact"])
def test_graph_frames_equal_eager_frames(env, kind):
    """The captured frame, replayed for a turning ring of cameras with eager
    frames and other device work in between, gives the eager images bit for
    bit on every replay."""
    nvgs, torch, _ = env
    sc = scene_of(kind)
    log(f"[graph] MLP {kind}")
    ctx = make_ctx(nvgs, sc)
    frames = [0, 7, 14]
    for f in frames:  # size the capacities from eager frames
        ctx.render(ring(sc, f), tile=16)
    wm = ctx.watermarks(reset=True)
    assert wm["max_splats"] > 0 and not wm["overflowed"]
    ctx.reserve(int(wm["max_splats"] * 1.5), int(wm["max_duplicates"] * 1.5))
    x = torch.randn(512, 512, device="cuda")
    for rep in range(3):
        for f in frames:
            cams = ring(sc, f)
            eager, se = ctx.render(cams, tile=16, stats=True)
            eager = eager.cpu().numpy()
            y = (x @ x).sum().item()  # unrelated device work between frames
            g = ctx.render(cams, tile=16, graph=True).clone()
            torch.cuda.synchronize()
            assert np.isfinite(y)
            same = np.array_equal(g.cpu().numpy(), eager)
            assert same, f"graph frame differs from the eager frame (replay {rep}, ring angle {f})"
            if rep == 0:
                _, sg = ctx.render(cams, tile=16, graph=True, stats=True)
                assert (sg["kept"], sg["duplicates"], sg["in_frustum"]) == \
                       (se["kept"], se["duplicates"], se["in_frustum"])
    wm = ctx.watermarks()
    log(f"[graph] watermarks {wm}")
    assert not wm["overflowed"]
    ctx.close()


def test_graph_frame_overflow_is_reported(env):
    """Capacities below the frame's needs: the persistent frame raises the
    overflow flag (E_CAPACITY with stats, sticky in the watermarks) and stays
    in bounds; after growing the capacities it matches the eager frame."""
    nvgs, torch, sc = env
    ctx = make_ctx(nvgs, sc)
    with pytest.raises(nvgs.NvgsError) as e:
        ctx.render(sc.cameras, tile=16, graph=True)
    assert e.value.status == nvgs.E_STATE  # no capacities yet
    ctx.reserve(4096, 4096)
    with pytest.raises(nvgs.NvgsError) as e:
        ctx.render(sc.cameras, tile=16, graph=True, stats=True)
    assert e.value.status == nvgs.E_CAPACITY
    wm = ctx.watermarks(reset=True)
    log(f"[overflow] watermarks after a clipped frame: {wm}")
    assert wm["overflowed"] and wm["max_splats"] > 4096
    # the entry count of a frame whose splats overflowed covers only the
    # splats that fit: grow from the watermarks until a frame fits
    for attempt in range(3):
        ctx.reserve(wm["max_splats"], wm["max_duplicates"])
        try:
            ctx.render(sc.cameras, tile=16, graph=True, stats=True)
            break
        except nvgs.NvgsError as e:
            assert e.status == nvgs.E_CAPACITY
            wm = ctx.watermarks(reset=True)
            log(f"[overflow] attempt {attempt}: {wm}")
    else:
        pytest.fail("capacities from the watermarks never fit the frame")
    assert not ctx.watermarks()["overflowed"]
    g = ctx.render(sc.cameras, tile=16, graph=True).clone()
    eager = ctx.render(sc.cameras, tile=16)
    same = np.array_equal(g.cpu().numpy(), eager.cpu().numpy())
    assert same, "graph frame differs from the eager frame"
    # the workspace by class: the classes add up, a splat costs 92 bytes and
    # an entry at least 16 (key and id, plus the shared ping-pong pair)
    _, st = ctx.render(sc.cameras, tile=16, stats=True)
    w = ctx.workspace_info()
    log(f"[workspace] {w}")
    assert w["total"] == st["workspace_bytes"]
    assert w["other"] >= 0 and w["debug"] == 0
    assert w["splats"] == 92 * w["splat_capacity"] and w["splat_capacity"] >= st["kept"]
    assert w["entries"] >= 16 * w["entry_capacity"] and w["entry_capacity"] >= st["duplicates"]
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_mlp_block_shapes_give_identical_results(env, prec):
    """Every MLP block shape computes each pair's logit in the same order:
    states and logits are bit-identical across shapes."""
    nvgs, torch, sc = env
    ctx = make_ctx(nvgs, sc)
    ref = None
    for gpw in (32, 64, 128):
        for segs in (1, 5, 16, 64):
            ctx.mlp_shape = (gpw, segs)
            st, lg = ctx.query_visibility(sc.cameras, precision=prec)
            cur = (st.cpu().numpy(), lg.cpu().numpy())
            if ref is None:
                ref = cur
            same_state = np.array_equal(cur[0], ref[0])
            same_logit = np.array_equal(cur[1].view(np.uint32), ref[1].view(np.uint32))
            assert same_state and same_logit, f"shape ({gpw}, {segs}) differs"
    ctx.close()


def test_autotuner(env):
    nvgs, torch, sc = env
    ctx = make_ctx(nvgs, sc)
    before = ctx.render(sc.cameras, tile=16, split=-1).cpu().numpy()
    tile, shape, table = ctx.autotune(sc.cameras, precision="bf16", reps=2)
    log(f"[tune] best tile {tile}, shape {shape}; {len(table)} measurements")
    assert tile in (8, 16, 32)
    assert shape[0] in (32, 64, 128) and shape[1] in (4, 8, 16, 32, 64)
    assert len(table) == 3 * 5 + 3 and all(r["ms"] > 0 for r in table)
    best_shape_ms = min(r["ms"] for r in table[:15])
    assert any(r["ms"] == best_shape_ms and (r["gaussians_per_wave"], r["segments_per_group"]) == shape
               for r in table[:15])
    # the tuned shape and tile change no pixel of the sequential composite (the
    # image depends on neither; with split lists a tile size cuts its lists at
    # other places, equal up to rounding)
    after = ctx.render(sc.cameras, tile=tile, split=-1).cpu().numpy()
    same = np.array_equal(before, after)
    assert same, "tuned frame differs"
    ctx.close()
