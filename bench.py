#!/usr/bin/env python3
"""Frame benchmark of the NVGS renderer on one MI355X.

One step is one full frame of the per-frame path (cull -> visibility MLP ->
compaction -> projection -> tile binning and sort -> compositing), run as the
library's persistent frame (one captured HIP graph replayed per frame, the
cameras uploaded before each replay).

--workload composed (default): the composed 1080p scene, 4 assets (torus,
sphere shell, box shell, helix tube) of 250,000 SH-degree-3 Gaussians each,
64 instances with random yaw, scale U(0.5, 2) and positions on a 40 x 40
ground plane, one camera, one width-64 FP32 visibility MLP per asset (run as
the split FP32 form: three BF16 matrix-core products per FP32 product, held
to the FP32 logit tolerance; the FP32-matrix-core form, BF16 and FP8 are
timed beside it).

--workload batched: 16 assets of log-uniform sizes in [50k, 1M] (SH 3),
1,024 instances with Zipf counts per asset on a 160 x 160 plane, 8 cameras at
1080p on a ring of radius 60 at height 15; the ring turns 1 degree per frame
over 360 frames for the p50 / p99 frame times.

Inputs are seeded synthetic stand-ins for the paper's scenes and are resident
in HBM before timing starts.  Before timing, each asset's MLP is trained by
the library on renderer-made labels (Sec. 3.1 recipe: Fibonacci views at
distances U(1.5, 20) with a random offset, 6 auxiliary views on a 5 degree
cone, class-frequency weighted BCE, BF16 forward/backward, Adam 1e-3,
batches of 65,536 pairs); `--mlp random` instead uses seeded weights with the
output bias set to keep 65% of the in-frustum pairs.  Tile size and MLP block
shape come from the library's autotuner unless --tile is given.

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# per queried pair: the two hidden layers and the output layer (layer 1 is
# computed once per Gaussian chunk and once per (camera, instance) segment)
FLOP_PER_QUERY = {64: 2 * (2 * 64 * 64 + 64), 128: 2 * (2 * 128 * 128 + 128)}
# compact form per queried pair: the per-pair part of layer 1 (4 inputs), layer 2 and the output
FLOP_PER_QUERY[32] = 2 * (4 * 32 + 32 * 32 + 32)
COMPACT_BO = 32 * 16 + 32 + 32 * 32 + 32 + 32  # index of the compact form's output bias
# dense MFMA peaks; the split FP32 form issues three BF16 products per FP32
# product, so its FP32-equivalent peak is a third of the BF16 one
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0, "fp32s": 2500.0 / 3}
MLP_ARITH = {"fp32": "FP32 operands on FP32 matrix cores",
             "fp32s": "FP32 MLP on BF16 matrix cores: each FP32 operand split into two BF16 parts, three products "
                      "per FP32 product, FP32 accumulation (logits within 1e-5 of the FP64 oracle's logit scale)",
             "bf16": "BF16 operands, FP32 accumulation", "fp8": "FP8 E4M3 operands, per-layer scales, FP32 accumulation"}
HBM_PEAK_GBS = 8000.0
VALU_LANE_OPS = 256 * 64 * 2.4e9          # non-packed FP32 lane-ops per second
BLEND_SLOTS_PER_TEST = 20
BLEND_PEAK_GTESTS = VALU_LANE_OPS / BLEND_SLOTS_PER_TEST / 1e9


def train_assets(ctx, sc, views=512, res=512, batch=65536, steps=5000, precision="bf16", lr=1e-3, seed=1,
                 weighting=1, aux=None, aux_deg=5.0, offset=None, recipe="workload", sampling="fibonacci",
                 fovy_deg=50.0):
    """Train each asset's visibility MLP on labels the renderer makes from
    `views` Fibonacci-sphere (or longitude-latitude) views of `fovy_deg`,
    each with `aux` auxiliary views on a cone of `aux_deg` degrees (one
    identity instance per asset), with class-frequency weighted BCE when
    `weighting`.  recipe "workload" (the differentiation workload's): distances
    U(1.5, 20), constant lr, no view offset and no auxiliary views unless
    given; recipe "paper" (Sec. 3.1, 4.1): the asset's Eq. 1 distance range
    (for the frequency form also its MLP's far clamp; the compact form
    normalises its distance input over it), the distance-scaled view offset,
    6 auxiliary views, batches of 2^19, lr 2e-3 with warm-up and decay to
    2e-4.  Returns per-asset summaries."""
    import torch
    import synth
    if aux is None:
        aux = 6 if recipe == "paper" else 0
    if offset is None:
        offset = 1.0 if recipe == "paper" else 0.0
    out = []
    for j, a in enumerate(sc.assets):
        d_lo, d_hi = 1.5, 20.0
        lr_final = 0.0
        if recipe == "paper":
            d_lo, d_hi = synth.eq1_range(a.name, fovy_deg=fovy_deg)
            if a.mlp.kind == 0:
                a.mlp.d_max = float(np.float32(d_hi))
                a.mlp.cam_scale = float(np.float32(1.0 / d_hi))  # keeps the encoded camera position in [-1, 1]
            batch, lr, lr_final = 1 << 19, 2e-3, 2e-4
        cams = synth.label_views(views, seed=synth.SEED_BASE + 500 + j, d_lo=d_lo, d_hi=d_hi, res=res,
                                 offset=offset, fovy_deg=fovy_deg, sampling=sampling,
                                 radius=synth.SHAPE_HALF_DIAG[a.name])
        params = torch.from_numpy(a.mlp.params.astype(np.float32).copy()).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        labels = ctx.make_labels(j, cams, aux=aux, aux_angle=math.radians(aux_deg))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if recipe == "paper":
            ctx.load_assets(sc.assets)  # the new far clamp
        curve = ctx.train_visibility(j, cams, params, labels=labels, batch=batch, steps=steps, precision=precision,
                                     lr=lr, seed=seed + j, weighting=weighting, lr_final=lr_final)
        t2 = time.perf_counter()
        a.mlp.params = params.cpu().numpy()
        visible = float(np.unpackbits(labels.cpu().numpy().view(np.uint8), bitorder="little").mean())
        out.append({"asset": a.name, "label_s": t1 - t0, "train_s": t2 - t1, "loss_first": float(curve[0]),
                    "loss_last100": float(curve[-100:].mean()), "label_visible_frac": visible})
        print(f"[train] {a.name} ({'compact' if a.mlp.kind == 1 else 'frequency'} form): labels {t1 - t0:.1f} s, "
              f"training {t2 - t1:.1f} s, loss {curve[0]:.4f} -> {curve[-100:].mean():.4f}", file=sys.stderr,
              flush=True)
    ctx.load_assets(sc.assets)
    ctx.set_instances(sc.instances)
    return out


def calibrate_keep(ctx, sc, frac, precision):
    """Set each asset's output bias so `frac` of its in-frustum pairs keep
    (threshold midway between neighbouring logits)."""
    _, lg = ctx.query_visibility(sc.cameras, precision=precision)
    lg = lg.cpu().numpy()
    off = sc.pair_offsets()
    for a_idx, a in enumerate(sc.assets):
        zs = [lg[:, off[i]:off[i + 1]] for i, inst in enumerate(sc.instances) if inst.asset == a_idx]
        z = np.concatenate([x.ravel() for x in zs]) if zs else np.zeros(0)
        z = np.sort(z[~np.isnan(z)])
        if len(z) < 2:
            continue
        k = int(np.clip(round((1 - frac) * len(z)), 1, len(z) - 1))
        p = a.mlp.params.copy()
        bo = COMPACT_BO if a.mlp.kind == 1 else -1  # the output bias
        p[bo] = np.float32(p[bo] - 0.5 * (z[k - 1] + z[k]))
        a.mlp.params = p
    ctx.load_assets(sc.assets)
    ctx.set_instances(sc.instances)


def time_frames(ctx, sc, steps, warmup, **kw):
    import torch
    for _ in range(warmup):
        ctx.render(sc.cameras, **kw)
    torch.cuda.synchronize()
    stage = None
    last = None
    t0 = time.perf_counter()
    for _ in range(steps):
        # stage times of the kernels a frame without statistics runs (the
        # compositing test count changes the compositing kernels)
        img, st = ctx.render(sc.cameras, stats=True, count_tests=False, **kw)
        ms = np.array(list(st["ms_stage"].values()))
        stage = ms if stage is None else stage + ms
        last = st
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    names = list(last["ms_stage"].keys())
    # one more frame for the compositing test count
    _, st_count = ctx.render(sc.cameras, stats=True, **kw)
    last = dict(last, blend_tests=st_count["blend_tests"])
    return (t1 - t0) / steps, dict(zip(names, (stage / steps).tolist())), last, img


def algorithmic_bytes(stage, st, sh_degree):
    """HBM bytes a memory-bound stage must move, per the method's data (the
    per-unit figures of the design notes): projection 56 B (SH 0) or 236 B
    (SH 3) of Gaussian read + a 48 B splat record written per kept splat; the
    depth sort of the splats 4 passes x 16 B (4 B key + 4 B id, read and
    written) per splat; binning 8 B per (tile, splat) entry written; the
    stable tile sort 2 passes x 16 B per entry."""
    if stage == "project":
        return st["kept"] * (44 + 12 * (sh_degree + 1) ** 2 + 48)
    if stage == "depth_sort":
        return st["kept"] * 64
    if stage == "bin":
        return st["duplicates"] * 8
    if stage == "tile_sort":
        return st["duplicates"] * 32
    return None


def implementation_bytes(stage, st, sh_degree, n_keys_tiles):
    """Bytes the kernels as built move: the projection's 48 B geometry record
    + SH row (rounded to 16 B) read and its 64 B compositing record, 8 B tile
    rectangle and 4 B depth key written; a radix pass 4 B histogram + 8 B read
    + 8 B written per key, the depth sort's last pass writing the 8 B
    rectangle and 4 B tile count it reads by id instead of the 4 B key (+16 B
    per splat); binning 28 B per splat (in-place count scan; emission: id,
    rectangle, offset) + 8 B per entry; the tile stage its radix passes + 4 B
    per entry for the ranges."""
    if stage == "project":
        return st["kept"] * (48 + 4 * (-(-3 * (sh_degree + 1) ** 2 // 4) * 4) + 76)
    if stage == "depth_sort":
        return st["kept"] * (4 * 20 + 16)
    if stage == "bin":
        return st["kept"] * 28 + st["duplicates"] * 8
    if stage == "tile_sort":
        passes = max(1, -(-max(1, int(n_keys_tiles - 1).bit_length()) // 8))
        return st["duplicates"] * (20 * passes + 4)
    return None


def stage_roof(stage, ms, st, width, precision, sh_degree, n_keys_tiles):
    """Roofline of one frame stage from its algorithmic work per launch: MLP
    FLOP per queried pair (layers 2, 3 and the output; layer 1's camera half
    is per (camera, instance) and its Gaussian half per 256-Gaussian chunk,
    both shared by many queries and not counted); fragment tests for the blend
    (about 20 VALU lane-slots each); algorithmic_bytes() for the memory-bound
    stages, with the implementation's own bytes beside them."""
    sec = ms * 1e-3
    if sec <= 0:
        return None
    if stage == "cull_mlp":
        a = st["queried"] * FLOP_PER_QUERY[width] / sec / 1e12
        p = MFMA_PEAK_TFLOPS[precision]
        return {"bound": "mfma", "achieved": a, "peak": p, "unit": "TFLOP/s", "frac": a / p}
    if stage == "blend":
        a = st["blend_tests"] / sec / 1e9
        return {"bound": "alu", "achieved": a, "peak": BLEND_PEAK_GTESTS, "unit": "Gtests/s",
                "frac": a / BLEND_PEAK_GTESTS}
    nb = algorithmic_bytes(stage, st, sh_degree)
    if nb is None:
        return None
    a = nb / sec / 1e9
    ib = implementation_bytes(stage, st, sh_degree, n_keys_tiles) / sec / 1e9
    return {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a / HBM_PEAK_GBS,
            "impl_achieved": ib, "impl_frac": ib / HBM_PEAK_GBS}


def roofline(stage_ms, st, width, precision, sh_degree, n_keys_tiles, workload="composed1080p"):
    """Roofline of the dominant kernel stage (see stage_roof), with the HBM
    traffic measured for its kernel on this workload when the committed
    counters match the source."""
    dom = max(stage_ms, key=stage_ms.get)
    r = {k: v for k, v in stage_roof(dom, stage_ms[dom], st, width, precision, sh_degree, n_keys_tiles).items()
         if not k.startswith("impl_")}
    r["traffic"] = measured_traffic(dom, workload)
    return dom, r


def stage_rooflines(stage_ms, st, width, precision, sh_degree, n_keys_tiles):
    out = {}
    for k, v in stage_ms.items():
        r = stage_roof(k, v, st, width, precision, sh_degree, n_keys_tiles)
        if r:
            out[k] = {"bound": r["bound"], "frac": round(r["frac"], 4), "achieved": round(r["achieved"], 2),
                      "unit": r["unit"]}
            if "impl_frac" in r:
                out[k]["impl_frac"] = round(r["impl_frac"], 4)
    return out


def measured_traffic(stage, workload):
    """HBM bytes per launch of the stage's kernel(s) on `workload` from the
    committed rocprofv3 counter summary, or None when none was measured for
    that workload or the kernel source changed since."""
    import hashlib
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[workload][stage]
        cur = hashlib.sha256(open(os.path.join(ROOT, t["source"]), "rb").read()).hexdigest()
        return t["fetch_bytes"] + t["write_bytes"] if cur == t["source_sha256"] else None
    except (OSError, KeyError, ValueError):
        return None


def workspace_report(ctx):
    """The context's device memory by class (GB) with the frame buffers'
    capacities and bytes per splat and per entry (peak VRAM of the frame
    beside the paper's VRAM figures, which are context, not a target)."""
    w = ctx.workspace_info()
    gb = {k: w[k] / 1e9 for k in ("total", "assets", "pairs", "splats", "entries", "tiles", "debug", "other")}
    return {"gb": gb, "splat_capacity": w["splat_capacity"], "entry_capacity": w["entry_capacity"],
            "bytes_per_splat": w["splats"] / max(1, w["splat_capacity"]),
            "bytes_per_entry": w["entries"] / max(1, w["entry_capacity"])}


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(sc, img_culled, every=1, every_1core=8):
    """The FP64 oracle timed on the host: on all cores, one full culled frame
    of the scene (every `every`-th instance if `every` > 1, the time then
    scaled by the pair-count ratio); on one core, every `every_1core`-th
    instance of that sample, scaled likewise.  The all-core run's unculled
    frame gives the PSNR of the GPU's culled image against the FP64
    reference."""
    import oracle
    import synth

    def timed(step, threads):
        used = oracle.set_threads(threads)
        sub = synth.Scene(assets=sc.assets, instances=sc.instances[::step], cameras=sc.cameras, tile=sc.tile)
        t0 = time.perf_counter()
        oracle.frame(sub, use_mlp=True, want_margin=False)
        dt = time.perf_counter() - t0
        return used, dt, sc.pairs_per_camera / sub.pairs_per_camera, len(sub.instances)

    res = f"{sc.cameras[0].width}x{sc.cameras[0].height}"
    used, dt, scale, ni = timed(every, 0)
    out = {"value": 1.0 / (dt * scale), "unit": "frames/s", "cores": used, "kind": "oracle",
           "sample": f"{ni} of {len(sc.instances)} instances, one full culled {res} frame in {dt:.1f} s on "
                     f"{used} threads" + (f", scaled x{scale:.1f} by pair count" if every > 1 else "")}
    used1, dt1, scale1, ni1 = timed(every * every_1core, 1)
    out["single_core"] = {"value": 1.0 / (dt1 * scale1), "unit": "frames/s", "cores": used1,
                          "sample": f"{ni1} of {len(sc.instances)} instances of the culled {res} frame in "
                                    f"{dt1:.1f} s on one thread, scaled x{scale1:.1f} by pair count"}
    out["host"] = host_cpu()
    oracle.set_threads(0)
    if every == 1:
        ref = oracle.frame(sc, use_mlp=False, want_margin=False)["images"][0]
        out["psnr_gpu_culled_vs_fp64_unculled_db"] = psnr(img_culled[0], ref)
    return out


def psnr(a, b):
    mse = float(np.mean((a.astype(np.float64) - b.astype(np.float64)) ** 2))
    return 100.0 if mse == 0 else min(100.0, 10 * math.log10(1.0 / mse))


def time_graph(ctx, cam_sets, steps, warmup, **kw):
    """Persistent frames: `warmup` untimed, then `steps` timed replays cycling
    through `cam_sets`; returns (wall seconds per frame, per-frame ms from
    HIP events on the context stream)."""
    import torch
    for i in range(warmup):
        ctx.render(cam_sets[i % len(cam_sets)], graph=True, **kw)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        evs[i][0].record(s)
        ctx.render(cam_sets[i % len(cam_sets)], graph=True, **kw)
        evs[i][1].record(s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = [a.elapsed_time(b) for a, b in evs]
    return (t1 - t0) / steps, per


def prepare(ctx, cam_sets, tile_arg, precision, reps=7, use_mlp_modes=(True, False)):
    """Autotune (unless a tile is given), then size the persistent frame's
    capacities from eager frames over the camera sets (10% headroom)."""
    tune = None
    if tile_arg == 0:
        tile, shape, table = ctx.autotune(cam_sets[0], precision=precision, reps=reps)
        tune = {"tile": tile, "mlp_shape": list(shape), "table": table}
    else:
        tile = tile_arg
    ctx.watermarks(reset=True)
    for cams in cam_sets:
        for um in use_mlp_modes:
            ctx.render(cams, tile=tile, precision=precision, use_mlp=um)
    wm = ctx.watermarks(reset=True)
    ctx.reserve(int(wm["max_splats"] * 1.1) + 4096, int(wm["max_duplicates"] * 1.1) + 4096)
    return tile, tune


def check_no_overflow(ctx):
    wm = ctx.watermarks(reset=True)
    if wm["overflowed"]:
        raise RuntimeError(f"a timed frame exceeded the reserved capacities: {wm}")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="composed", choices=["composed", "batched", "sweep", "ablation", "precision", "train"],
                    help="sweep: composed scene at several camera distances, SH 3 and SH 0, culled / unculled / "
                         "radius-clipped")
    ap.add_argument("--det-clip", type=float, default=0.1, help="sweep, ablation: radius-clipping threshold (px^4)")
    ap.add_argument("--tile", type=int, default=0, help="8, 16, 32, or 0 to autotune (tile and MLP block shape)")
    ap.add_argument("--precision", default=None,
                    help="MLP precision: fp32s (FP32 via split BF16 products), fp32, bf16, fp8 (default fp32s "
                         "composed, bf16 batched)")
    ap.add_argument("--mlp", default="trained", choices=["trained", "random"],
                    help="trained: per-asset MLPs trained on renderer labels; random: seeded weights with the "
                         "output bias set to keep --keep of the in-frustum pairs")
    ap.add_argument("--train-steps", type=int, default=5000)
    ap.add_argument("--views", type=int, default=2000, help="label views per asset")
    ap.add_argument("--recipe", default="paper", choices=["workload", "paper"],
                    help="training recipe: workload (U(1.5, 20) views, batch 65,536, lr 1e-3) or paper (Eq. 1 "
                         "range, batch 2^19, lr 2e-3 -> 2e-4 with warm-up)")
    ap.add_argument("--keep", type=float, default=0.65)
    ap.add_argument("--n", type=int, default=250000)
    ap.add_argument("--frames", type=int, default=360, help="batched: ring positions (1 degree apart)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compact", action="store_true", help="composed: skip the compact-form comparison")
    ap.add_argument("--aligned", action="store_true",
                    help="composed, sweep, ablation: flat surface-aligned Gaussians instead of random orientations")
    ap.add_argument("--compact-steps", type=int, default=0,
                    help="training steps of the compact form (0: --train-steps)")
    ap.add_argument("--extra-precisions", default="fp32,bf16,fp8",
                    help="comma list of MLP forms timed beside the headline one")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many bytes (calibrates HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.copy_probe:
        import torch
        a = torch.empty(args.copy_probe // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported: splitting a frame across "
              "GPUs (by camera, or by screen band after projection) is designed but not built", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        return main_batched(args)
    if args.workload == "sweep":
        return main_sweep(args)
    if args.workload == "ablation":
        return main_ablation(args)
    if args.workload == "precision":
        return main_precision(args)
    if args.workload == "train":
        return main_train(args)
    import torch
    import paper_2511_19202_amd as nvgs
    import synth

    prec = args.precision or "fp32s"
    sc = synth.scene_composed(n_per_asset=args.n, aligned=args.aligned)
    ctx = nvgs.Context(0)
    ctx.load_assets(sc.assets)
    ctx.set_instances(sc.instances)
    training = None
    if args.mlp == "trained":
        training = train_assets(ctx, sc, views=args.views, steps=args.train_steps, recipe=args.recipe)
    else:
        calibrate_keep(ctx, sc, args.keep, prec)
    tile, tune = prepare(ctx, [sc.cameras], args.tile, prec)
    kw = dict(tile=tile, precision=prec)
    # headline: persistent frames, culled and unculled
    t_c, per_c = time_graph(ctx, [sc.cameras], args.steps, args.warmup, use_mlp=True, **kw)
    t_u, per_u = time_graph(ctx, [sc.cameras], args.steps, args.warmup, use_mlp=False, **kw)
    check_no_overflow(ctx)
    # per-stage kernel times and counts: eager frames with HIP stage events
    _, stage_c, st_c, img_c = time_frames(ctx, sc, max(5, args.steps // 5), 2, use_mlp=True, **kw)
    img_c = img_c.cpu().numpy()
    _, stage_u, st_u, img_u = time_frames(ctx, sc, max(5, args.steps // 5), 2, use_mlp=False, **kw)
    img_u = img_u.cpu().numpy()
    g_c = ctx.render(sc.cameras, graph=True, use_mlp=True, **kw).cpu().numpy()
    graph_equals_eager = bool(np.array_equal(g_c, img_c))

    width = sc.assets[0].mlp.width
    cam0 = sc.cameras[0]
    nkt = len(sc.cameras) * (-(-cam0.width // tile)) * (-(-cam0.height // tile))
    dom, roof = roofline(stage_c, st_c, width, prec, sc.assets[0].sh_degree, nkt)
    stage_roofs = stage_rooflines(stage_c, st_c, width, prec, sc.assets[0].sh_degree, nkt)
    extra = {}
    for p2 in [p for p in args.extra_precisions.split(",") if p]:
        try:
            t_p, _ = time_graph(ctx, [sc.cameras], args.steps, args.warmup, use_mlp=True, tile=tile, precision=p2)
            check_no_overflow(ctx)
            _, stage_p, st_p, img_p = time_frames(ctx, sc, 5, 1, use_mlp=True, tile=tile, precision=p2)
            extra[p2] = {"fps": 1.0 / t_p, "ms_cull_mlp": stage_p["cull_mlp"], "mlp_arith": MLP_ARITH.get(p2),
                         "psnr_vs_headline_culled_db": psnr(img_p.cpu().numpy(), img_c),
                         "psnr_vs_unculled_db": psnr(img_p.cpu().numpy(), img_u),
                         "kept": st_p["kept"]}
        except Exception as e:  # report, do not hide
            extra[p2] = {"error": str(e)}
    fps = 1.0 / t_c
    out = {
        "metric": "1080p FPS + visibility-MLP queries/s, culled vs unculled, PSNR vs FP64 oracle",
        "value": fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_c,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "composed-1080p: 4 assets x 250k SH3 Gaussians, 64 instances, 1 camera, "
                               "width-64 MLP per asset",
                   "gaussian_orientation": "surface-aligned discs" if args.aligned else "random",
                   "gaussians_stored": sum(a.n for a in sc.assets), "instances": len(sc.instances),
                   "pairs": st_c["pairs"], "resolution": "1920x1080", "mlp_precision": prec,
                   "mlp_arith": MLP_ARITH.get(prec),
                   "tile": tile, "mlp_shape": list(ctx.mlp_shape), "autotune": tune, "mlp": args.mlp,
                   "keep_target": args.keep if args.mlp == "random" else None, "frame": "persistent (HIP graph)"},
        "fps_unculled": 1.0 / t_u,
        "frame_ms_p50": float(np.percentile(per_c, 50)), "frame_ms_p99": float(np.percentile(per_c, 99)),
        "frame_ms_p50_unculled": float(np.percentile(per_u, 50)),
        "mlp_queries_per_s": st_c["queried"] / (stage_c["cull_mlp"] * 1e-3),
        "gaussians_per_s": st_c["pairs"] / t_c,
        "psnr_culled_vs_unculled_db": psnr(img_c, img_u),
        "graph_frame_equals_eager_frame": graph_equals_eager,
        "in_frustum": st_c["in_frustum"], "queried": st_c["queried"], "kept": st_c["kept"],
        "duplicates": st_c["duplicates"], "duplicates_unculled": st_u["duplicates"],
        "blend_tests": st_c["blend_tests"], "blend_tests_unculled": st_u["blend_tests"],
        "compositing_items": st_c["blend_items"], "compositing_items_unculled": st_u["blend_items"],
        "chunk_len": st_c["chunk_len"], "chunk_len_unculled": st_u["chunk_len"],
        "ms_stage": stage_c, "ms_stage_unculled": stage_u,
        "dominant_kernel": dom,
        "roofline": roof,
        "stage_rooflines": stage_roofs,
        "precisions": extra,
        "workspace_bytes": st_c["workspace_bytes"],
        "workspace": workspace_report(ctx),
        "keep_frac_of_in_frustum": st_c["kept"] / max(1, st_c["in_frustum"]),
        "training": training,
    }
    if not args.no_compact:
        out["compact_form"] = compact_report(ctx, sc, args, img_u)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, img_c)
    print(json.dumps(out), flush=True)
    ctx.close()


def compact_assets(sc, fovy_deg=50.0):
    """The scene's assets with the paper's compact MLP form (Sec. 3.2):
    seeded weights, distance input normalised over the asset's Eq. 1 range."""
    import synth
    return [synth.make_compact(a, synth.SEED_BASE + 700 + j, *synth.eq1_range(a.name, fovy_deg=fovy_deg))
            for j, a in enumerate(sc.assets)]


def compact_report(ctx, sc, args, img_u):
    """The same frame with each asset's MLP in the paper's compact form,
    trained with the same recipe (or calibrated like the headline form): FPS,
    MLP stage time and queries/s, PSNR against the unculled frame, in FP32 and
    with a BF16 second layer."""
    import copy
    sc2 = copy.copy(sc)
    sc2.assets = compact_assets(sc)
    ctx.load_assets(sc2.assets)
    ctx.set_instances(sc2.instances)
    training = None
    if args.mlp == "trained":
        training = train_assets(ctx, sc2, views=args.views, steps=args.compact_steps or args.train_steps,
                                recipe=args.recipe)
    else:
        calibrate_keep(ctx, sc2, args.keep, "fp32")
    tile, tune = prepare(ctx, [sc2.cameras], args.tile, "fp32")
    rep = {"tile": tile, "mlp_shape": list(ctx.mlp_shape), "autotune": tune, "training": training,
           "params_per_asset": int(sc2.assets[0].mlp.params.size)}
    for p in ("fp32", "bf16"):
        t, per = time_graph(ctx, [sc2.cameras], args.steps, args.warmup, use_mlp=True, tile=tile, precision=p)
        check_no_overflow(ctx)
        _, stage, st, img = time_frames(ctx, sc2, max(5, args.steps // 5), 2, use_mlp=True, tile=tile, precision=p)
        rep[p] = {"fps": 1.0 / t, "frame_ms_p50": float(np.percentile(per, 50)),
                  "frame_ms_p99": float(np.percentile(per, 99)), "ms_stage": stage,
                  "mlp_queries_per_s": st["queried"] / (stage["cull_mlp"] * 1e-3),
                  "psnr_culled_vs_unculled_db": psnr(img.cpu().numpy(), img_u), "queried": st["queried"],
                  "kept": st["kept"], "keep_frac_of_in_frustum": st["kept"] / max(1, st["in_frustum"]),
                  "workspace_bytes": st["workspace_bytes"]}
    # restore the headline form
    ctx.load_assets(sc.assets)
    ctx.set_instances(sc.instances)
    return rep


def main_ablation(args):
    """A synthetic analogue of the paper's ablation (Sec. 4.3): compact MLPs
    trained on views of 60 degree FoV, rendered by a 20 degree camera at six
    distances along one ray; variants add, in order, Fibonacci instead of
    longitude-latitude view sampling, the random view offset, auxiliary
    views, the FoV correction of Eq. 2 (without it the renderer feeds the
    uncorrected distance) and radius clipping.  Per variant: FPS at the
    largest distance, PSNR and 1 - SSIM against the unculled frame averaged
    over the distances, and the peak frame workspace."""
    import copy
    import torch
    import paper_2511_19202_amd as nvgs
    import synth

    prec = args.precision or "fp32"
    f_train, fov_r = 60.0, 20.0
    sc = synth.scene_composed(n_per_asset=args.n, aligned=args.aligned)
    sc.assets = compact_assets(sc, fovy_deg=f_train)
    ft = float(np.float32(0.5 * 512 / math.tan(math.radians(f_train) / 2)))
    for a in sc.assets:
        a.mlp.train_focal = ft
    base = sc.cameras[0]
    # the narrow camera backed off so that it frames the composed plane as the 50 degree one does
    back = math.tan(math.radians(25.0)) / math.tan(math.radians(fov_r / 2))
    factors = (1.0, 1.5, 2.0, 3.0, 4.0, 6.0)
    cams = [synth.camera(np.asarray(base.pos, np.float64) * back * f, fovy_deg=fov_r, width=base.width,
                         height=base.height) for f in factors]
    f_r = 0.5 * base.height / math.tan(float(np.float32(math.radians(fov_r))) / 2)
    ctx = nvgs.Context(0)
    ctx.load_assets(sc.assets)
    ctx.set_instances(sc.instances)

    def size_for(cam, **kw):
        ctx.watermarks(reset=True)
        ctx.render([cam], tile=8, precision=prec, **kw)
        wm = ctx.watermarks(reset=True)
        ctx.reserve(int(wm["max_splats"] * 1.1) + 4096, int(wm["max_duplicates"] * 1.1) + 4096)

    # unculled references and their FPS (the same for every variant)
    ref, fps_u = [], []
    for cam in cams:
        ref.append(ctx.render([cam], tile=8, precision=prec, use_mlp=False).cpu().numpy()[0])
        size_for(cam, use_mlp=False)
        t, _ = time_graph(ctx, [[cam]], 20, 3, tile=8, precision=prec, use_mlp=False)
        fps_u.append(1.0 / t)
    trainings = {"longlat": dict(sampling="longlat", offset=0.0, aux=0),
                 "fibonacci": dict(offset=0.0, aux=0),
                 "offset": dict(offset=1.0, aux=0),
                 "aux": dict(offset=1.0, aux=6)}
    variants = [("LongLat sampling", "longlat", False, 0.0), ("Fibonacci sampling", "fibonacci", False, 0.0),
                ("+ random offset", "offset", False, 0.0), ("+ auxiliary views", "aux", False, 0.0),
                ("full (+ FoV correction)", "aux", True, 0.0), ("+ radius clipping", "aux", True, args.det_clip)]
    trained = {}
    rows = []
    init = [a.mlp.params for a in sc.assets]  # every variant trains from the same seeded weights
    for name, tkey, fov_corr, clip in variants:
        if tkey not in trained:
            scv = copy.copy(sc)
            scv.assets = [copy.copy(a) for a in sc.assets]
            for a, p in zip(scv.assets, init):
                a.mlp = copy.copy(a.mlp)
                a.mlp.params = p
                a.mlp.train_focal = ft
            ctx.load_assets(scv.assets)
            ctx.set_instances(scv.instances)
            t0 = time.perf_counter()
            train_assets(ctx, scv, views=args.views, steps=args.compact_steps or args.train_steps, recipe="paper",
                         fovy_deg=f_train, **trainings[tkey])
            trained[tkey] = ([a.mlp.params for a in scv.assets], time.perf_counter() - t0)
            print(f"[ablation] trained '{tkey}' in {trained[tkey][1]:.1f} s", file=sys.stderr, flush=True)
        for a, p in zip(sc.assets, trained[tkey][0]):
            a.mlp.params = p
            # without the correction the renderer's own focal length stands in for the training one
            a.mlp.train_focal = ft if fov_corr else float(np.float32(f_r))
        ctx.load_assets(sc.assets)
        ctx.set_instances(sc.instances)
        per_d = []
        for cam, r in zip(cams, ref):
            img, st = ctx.render([cam], tile=8, precision=prec, det_clip=clip, stats=True)
            img = img.cpu().numpy()[0]
            size_for(cam, det_clip=clip)
            t, _ = time_graph(ctx, [[cam]], 20, 3, tile=8, precision=prec, det_clip=clip)
            check_no_overflow(ctx)
            per_d.append({"distance": float(np.linalg.norm(cam.pos)), "fps": 1.0 / t, "psnr_db": psnr(img, r),
                          "ssim": ssim(img, r), "kept": st["kept"], "in_frustum": st["in_frustum"],
                          "workspace_gb": st["workspace_bytes"] / 1e9})
        row = {"variant": name, "fps_at_max_distance": per_d[-1]["fps"],
               "psnr_mean_db": float(np.mean([x["psnr_db"] for x in per_d])),
               "one_minus_ssim_mean": float(np.mean([1 - x["ssim"] for x in per_d])),
               "workspace_gb_peak": max(x["workspace_gb"] for x in per_d), "per_distance": per_d}
        rows.append(row)
        print(f"[ablation] {name}: {row['fps_at_max_distance']:.1f} FPS at the largest distance, "
              f"PSNR {row['psnr_mean_db']:.2f} dB, 1-SSIM {row['one_minus_ssim_mean']:.4f}, "
              f"{row['workspace_gb_peak']:.2f} GB", file=sys.stderr, flush=True)
    print(json.dumps({"workload": "ablation: composed scene, compact MLPs trained at 60 deg FoV, 20 deg camera "
                                  "at 6 distances", "mlp_precision": prec, "det_clip": args.det_clip,
                      "unculled_fps": fps_u, "distances": [float(np.linalg.norm(c.pos)) for c in cams],
                      "training_s": {k: v[1] for k, v in trained.items()}, "rows": rows}), flush=True)
    ctx.close()


def main_batched(args):
    """8 cameras x 1080p in one persistent frame; the ring turns 1 degree per
    frame; p50 / p99 over the timed frames."""
    import torch
    import paper_2511_19202_amd as nvgs
    import synth

    prec = args.precision or "bf16"
    sc = synth.scene_batched()
    ctx = nvgs.Context(0)
    ctx.load_assets(sc.assets)
    ctx.set_instances(sc.instances)
    print(f"[batched] {len(sc.assets)} assets, {sum(a.n for a in sc.assets)} Gaussians stored, "
          f"{len(sc.instances)} instances, {sc.pairs_per_camera} pairs per camera", file=sys.stderr, flush=True)
    training = None
    if args.mlp == "trained":
        training = train_assets(ctx, sc, views=args.views, steps=args.train_steps, recipe=args.recipe)
        print("[batched] trained", file=sys.stderr, flush=True)
    else:
        calibrate_keep(ctx, sc, args.keep, prec)
    c0 = sc.cameras[0]
    rings = [synth.ring_cameras(len(sc.cameras), f, res=(c0.width, c0.height)) for f in range(args.frames)]
    # the ring repeats every 360 / 8 = 45 degrees: size from eager frames over one period
    period = [rings[f] for f in range(0, min(45, args.frames), 5)]
    tile, tune = prepare(ctx, period, args.tile, prec, use_mlp_modes=(True,))
    print(f"[batched] tile {tile}, MLP shape {ctx.mlp_shape}", file=sys.stderr, flush=True)
    kw = dict(tile=tile, precision=prec, use_mlp=True)
    steps = max(args.steps, args.frames)
    t_f, per = time_graph(ctx, rings, steps, args.warmup, **kw)
    check_no_overflow(ctx)
    _, stage, st, img = time_frames(ctx, sc, 3, 1, **kw)
    # culled vs unculled on two cameras of the first ring position (GPU images;
    # the unculled 8-camera frame would hold ~2.5e9 tile entries)
    ic = img.cpu().numpy()[:2]
    iu = ctx.render(sc.cameras[:2], tile=tile, precision=prec, use_mlp=False).cpu().numpy()
    psnrs = [psnr(ic[k], iu[k]) for k in range(2)]
    width = sc.assets[0].mlp.width
    cam0 = sc.cameras[0]
    nkt = len(sc.cameras) * (-(-cam0.width // tile)) * (-(-cam0.height // tile))
    dom, roof = roofline(stage, st, width, prec, sc.assets[0].sh_degree, nkt, workload="batched8x1080p")
    stage_roofs = stage_rooflines(stage, st, width, prec, sc.assets[0].sh_degree, nkt)
    C = len(sc.cameras)
    out = {
        "metric": "1080p FPS + visibility-MLP queries/s, culled vs unculled, PSNR vs FP64 oracle",
        "value": C / t_f,
        "unit": "1080p camera frames/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_f,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched-8cam-1080p: 16 assets (50k-1M log-uniform, SH3), 1024 Zipf instances, "
                               "8 ring cameras turning 1 deg per frame",
                   "gaussians_stored": sum(a.n for a in sc.assets), "instances": len(sc.instances),
                   "pairs": st["pairs"], "cameras": C, "resolution": "1920x1080", "mlp_precision": prec,
                   "tile": tile, "mlp_shape": list(ctx.mlp_shape), "autotune": tune, "mlp": args.mlp,
                   "frame": "persistent (HIP graph)"},
        "frame_ms_p50": float(np.percentile(per, 50)), "frame_ms_p99": float(np.percentile(per, 99)),
        "frame_ms_mean": float(np.mean(per)),
        "mlp_queries_per_s": st["queried"] / (stage["cull_mlp"] * 1e-3),
        "gaussians_per_s": st["pairs"] / t_f,
        "psnr_culled_vs_unculled_db_cameras_0_1": psnrs,
        "in_frustum": st["in_frustum"], "queried": st["queried"], "kept": st["kept"],
        "duplicates": st["duplicates"], "blend_tests": st["blend_tests"], "ms_stage": stage,
        "dominant_kernel": dom, "roofline": roof,
        "stage_rooflines": stage_roofs, "workspace_bytes": st["workspace_bytes"],
        "workspace": workspace_report(ctx),
        "training": training,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batched(sc)
    print(json.dumps(out), flush=True)
    ctx.close()


def ssim(a, b):
    """Mean SSIM over the RGB channels (Gaussian window sigma 1.5, constants
    of the usual definition, data range 1)."""
    from scipy.ndimage import gaussian_filter
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    out = []
    for ch in range(3):
        x, y = a[..., ch].astype(np.float64), b[..., ch].astype(np.float64)
        mx, my = gaussian_filter(x, 1.5), gaussian_filter(y, 1.5)
        sxx = gaussian_filter(x * x, 1.5) - mx * mx
        syy = gaussian_filter(y * y, 1.5) - my * my
        sxy = gaussian_filter(x * y, 1.5) - mx * my
        out.append(np.mean(((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))))
    return float(np.mean(out))


def main_sweep(args):
    """FPS against camera distance (the camera moved along its ray to the
    origin), for SH degree 3 and the same scene at SH degree 0, culled by the
    trained MLP, unculled, and culled with radius clipping; PSNR / SSIM of
    each culled image against the unculled one and the frame workspace."""
    import copy
    import torch
    import paper_2511_19202_amd as nvgs
    import synth

    prec = args.precision or "fp32s"
    sc = synth.scene_composed(n_per_asset=args.n, aligned=args.aligned)
    ctx = nvgs.Context(0)
    ctx.load_assets(sc.assets)
    ctx.set_instances(sc.instances)
    if args.mlp == "trained":
        train_assets(ctx, sc, views=args.views, steps=args.train_steps, recipe=args.recipe)
    else:
        calibrate_keep(ctx, sc, args.keep, prec)
    sc0 = copy.copy(sc)
    sc0.assets = []
    for a in sc.assets:  # the same Gaussians with only the degree-0 coefficients
        b = copy.copy(a)
        b.sh = np.ascontiguousarray(a.sh[:3])
        b.sh_degree = 0
        sc0.assets.append(b)
    base = sc.cameras[0]
    rows = []
    for label, scene in (("sh3", sc), ("sh0", sc0)):
        ctx.load_assets(scene.assets)
        ctx.set_instances(scene.instances)
        for fct in (0.5, 0.75, 1.0, 1.5, 2.0, 3.0, 4.0):
            cam = synth.camera(np.asarray(base.pos, np.float64) * fct, fovy_deg=math.degrees(base.fovy),
                               width=base.width, height=base.height)
            cams = [cam]
            row = {"sh": label, "distance": float(np.linalg.norm(cam.pos))}
            imgs = {}
            for mode, kw in (("culled", dict(use_mlp=True)), ("unculled", dict(use_mlp=False)),
                             ("culled_clip", dict(use_mlp=True, det_clip=args.det_clip))):
                img, st = ctx.render(cams, tile=8, precision=prec, stats=True, **kw)
                imgs[mode] = img.cpu().numpy()[0]
                ctx.watermarks(reset=True)
                ctx.render(cams, tile=8, precision=prec, **kw)
                wm = ctx.watermarks(reset=True)
                ctx.reserve(int(wm["max_splats"] * 1.1) + 4096, int(wm["max_duplicates"] * 1.1) + 4096)
                t, per = time_graph(ctx, [cams], 20, 3, tile=8, precision=prec, **kw)
                check_no_overflow(ctx)
                row[mode] = {"fps": 1.0 / t, "kept": st["kept"], "entries": st["duplicates"],
                             "workspace_gb": st["workspace_bytes"] / 1e9}
            for mode in ("culled", "culled_clip"):
                row[mode]["psnr_vs_unculled_db"] = psnr(imgs[mode], imgs["unculled"])
                row[mode]["ssim_vs_unculled"] = ssim(imgs[mode], imgs["unculled"])
            rows.append(row)
            print(f"[sweep] {label} d={row['distance']:.1f}: culled {row['culled']['fps']:.1f} FPS, unculled "
                  f"{row['unculled']['fps']:.1f}, clipped {row['culled_clip']['fps']:.1f}", file=sys.stderr, flush=True)
    print(json.dumps({"workload": "sweep: composed-1080p at 7 camera distances, SH 3 and SH 0",
                      "mlp_precision": prec, "det_clip": args.det_clip, "rows": rows}), flush=True)
    ctx.close()


def main_precision(args):
    """The precision form on the tiny scene (20k-Gaussian torus, 256^2, one
    camera): MLP widths 64 and 128 in FP32, BF16 and FP8 -- FPS, the keep
    flip rate against the FP64 MLP and the PSNR against the unculled FP64
    render (both from the oracle, in the cpu_baseline leg) -- and the MLP
    kernel alone on the composed scene's 16M pairs, where it fills the GPU:
    queries/s and the fraction of the MFMA peak of each precision.  Both
    widths are trained with the differentiation workload's recipe at 20k
    Gaussians (unless --mlp random: seeded weights with the output bias set
    to keep 65 % of the in-frustum pairs)."""
    import torch
    import paper_2511_19202_amd as nvgs
    import synth

    precs = ("fp32", "fp32s", "bf16", "fp8")
    tiny_rows, keep = [], {}
    for W in (64, 128):
        sc = synth.scene_tiny(n=20000, res=256, width=W)
        ctx = nvgs.Context(0)
        ctx.load_assets(sc.assets)
        ctx.set_instances(sc.instances)
        if args.mlp == "trained":
            train_assets(ctx, sc, views=512, res=512, batch=65536, steps=args.train_steps, recipe="workload")
            how = "trained"
        else:
            calibrate_keep(ctx, sc, args.keep, "fp32")
            how = "seeded, 65 % kept"
        row = {"width": W, "mlp": how}
        for prec in precs + ("unculled",):
            kw = dict(tile=16, precision="fp32" if prec == "unculled" else prec, use_mlp=prec != "unculled")
            ctx.watermarks(reset=True)
            img = ctx.render(sc.cameras, **kw).cpu().numpy()[0]
            wm = ctx.watermarks(reset=True)
            ctx.reserve(int(wm["max_splats"] * 1.1) + 4096, int(wm["max_duplicates"] * 1.1) + 4096)
            t, per = time_graph(ctx, [sc.cameras], args.steps, args.warmup, **kw)
            r = {"fps": 1.0 / t, "frame_ms_p50": float(np.percentile(per, 50))}
            if prec != "unculled":
                _, lg = ctx.query_visibility(sc.cameras, precision=prec)
                keep[(W, prec)] = (lg.cpu().numpy()[0].astype(np.float64), img)
            row[prec] = r
        tiny_rows.append((sc, row))
        ctx.close()
        print(f"[precision] tiny W={W}: " + ", ".join(f"{p} {row[p]['fps']:.0f} FPS" for p in precs + ("unculled",)),
              file=sys.stderr, flush=True)
    # the MLP kernel alone at the composed scene's 16M pairs
    big = []
    for W in (64, 128):
        sc = synth.scene_composed(n_per_asset=args.n, width=W)
        ctx = nvgs.Context(0)
        ctx.load_assets(sc.assets)
        ctx.set_instances(sc.instances)
        calibrate_keep(ctx, sc, args.keep, "fp32")
        for prec in precs:
            _, stage, st, _ = time_frames(ctx, sc, 5, 2, tile=8, precision=prec)
            sec = stage["cull_mlp"] * 1e-3
            tf = st["queried"] * FLOP_PER_QUERY[W] / sec / 1e12
            big.append({"width": W, "precision": prec, "ms": stage["cull_mlp"], "queried": st["queried"],
                        "queries_per_s": st["queried"] / sec, "tflops": tf, "peak_tflops": MFMA_PEAK_TFLOPS[prec],
                        "frac": tf / MFMA_PEAK_TFLOPS[prec]})
        ctx.close()
    out = {"workload": "precision: tiny scene (20k torus, 256^2) at MLP widths 64/128 in FP32/BF16/FP8; the MLP "
                       "kernel on the composed scene's 16M pairs",
           "tiny": [row for _, row in tiny_rows], "mlp_kernel_composed": big}
    if not args.no_cpu_baseline:
        import oracle
        cb = []
        for sc, row in tiny_rows:
            t0 = time.perf_counter()
            _, olg = oracle.query(sc)
            ref = oracle.frame(sc, use_mlp=False, want_margin=False)["images"][0]
            dt = time.perf_counter() - t0
            olg = olg[0]
            for prec in precs:
                lg, img = keep[(row["width"], prec)]
                q = ~np.isnan(olg) & ~np.isnan(lg)
                row[prec]["flip_rate_vs_fp64_mlp"] = float(np.mean((lg[q] >= 0) != (olg[q] >= 0)))
                row[prec]["psnr_vs_fp64_unculled_db"] = psnr(img, ref)
            cb.append({"width": row["width"], "seconds": dt})
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = {"value": 2.0 / sum(c["seconds"] for c in cb), "unit": "frames/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "FP64 MLP query and unculled render of the tiny scene at widths 64 and 128"}
    print(json.dumps(out), flush=True)


def main_train(args):
    """The differentiation workload: one 500k-Gaussian SH3 torus; labels
    rendered by the library from 512 views at distances U(1.5, 20) (512^2);
    5,000 BF16 training steps of 65,536 (Gaussian, view) pairs, FP32 master
    weights, Adam 1e-3, class-balanced BCE; then recall and precision of the
    trained MLP's keep decision against the renderer's labels on 64 held-out
    views, and its frame on one of them against the unculled frame.  The
    gradient itself is checked against the FP64 oracle and central
    differences by the tests."""
    import torch
    import paper_2511_19202_amd as nvgs
    import synth

    sc = synth.scene_train()
    a = sc.assets[0]
    ctx = nvgs.Context(0)
    ctx.load_assets(sc.assets)
    ctx.set_instances(sc.instances)
    views = synth.label_views(512, seed=synth.SEED_BASE + 5, d_lo=1.5, d_hi=20.0, res=512)
    hold = synth.label_views(64, seed=synth.SEED_BASE + 55, d_lo=1.5, d_hi=20.0, res=512)
    params = torch.from_numpy(a.mlp.params.astype(np.float32).copy()).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    labels = ctx.make_labels(0, views)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    curve = ctx.train_visibility(0, views, params, labels=labels, batch=65536, steps=args.train_steps,
                                 precision="bf16", lr=1e-3, seed=7, weighting=1)
    t2 = time.perf_counter()
    print(f"[train] labels {t1 - t0:.2f} s, {args.train_steps} steps in {t2 - t1:.2f} s, loss {curve[0]:.4f} -> "
          f"{curve[-100:].mean():.4f}", file=sys.stderr, flush=True)
    a.mlp.params = params.cpu().numpy()
    ctx.load_assets(sc.assets)
    ctx.set_instances(sc.instances)
    hl = ctx.make_labels(0, hold).cpu().numpy().view(np.uint32)
    vis = np.unpackbits(hl.view(np.uint8).reshape(len(hold), -1), axis=1, bitorder="little")[:, :a.n].astype(bool)
    st, _ = ctx.query_visibility(hold, want_logits=False)
    kept = st.cpu().numpy() == 2
    tp = float(np.sum(kept & vis))
    recall = tp / max(1.0, float(vis.sum()))
    prec = tp / max(1.0, float(kept.sum()))
    cam = hold[0]
    ic = ctx.render([cam], tile=16).cpu().numpy()[0]
    iu = ctx.render([cam], tile=16, use_mlp=False).cpu().numpy()[0]
    ctx.close()
    n_samples = 65536 * args.train_steps
    out = {"workload": "differentiation: 500k-Gaussian SH3 torus, labels from 512 views at U(1.5, 20), 512^2; BF16 "
                       "training, batches of 65,536, Adam 1e-3, class-balanced BCE",
           "label_views": len(views), "label_s": t1 - t0, "train_steps": args.train_steps, "train_s": t2 - t1,
           "samples_per_s": n_samples / (t2 - t1), "loss_first": float(curve[0]),
           "loss_last100": float(curve[-100:].mean()), "visible_frac_labels": float(vis.mean()),
           "holdout_views": len(hold), "holdout_recall": recall, "holdout_precision": prec,
           "holdout_kept_frac": float(kept.mean()),
           "psnr_culled_vs_unculled_db_holdout0": psnr(ic, iu)}
    print(json.dumps(out), flush=True)


def cpu_baseline_batched(sc, every=16):
    """The FP64 oracle on a deterministic subsample (camera 0, every 16th
    instance), its time scaled by the pair-count ratio to the whole frame."""
    import oracle
    import synth
    sub = synth.Scene(assets=sc.assets, instances=sc.instances[::every], cameras=sc.cameras[:1], tile=sc.tile)
    t0 = time.perf_counter()
    oracle.frame(sub, use_mlp=True, want_margin=False)
    dt = time.perf_counter() - t0
    scale = len(sc.cameras) * sc.pairs_per_camera / sub.pairs_per_camera
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": len(sc.cameras) / (dt * scale), "unit": "1080p camera frames/s", "cores": threads,
            "kind": "oracle", "extrapolated": True,
            "sample": f"camera 0 and {len(sub.instances)} of {len(sc.instances)} instances in {dt:.1f} s, "
                      f"scaled x{scale:.1f} by pair count to the 8-camera frame"}


if __name__ == "__main__":
    main()
