"""Test scenes: synthetic inputs with the MLP's output bias set so that a
given fraction of in-frustum pairs is kept (the oracle computes the logits)."""
import numpy as np

import oracle
import synth


def calibrate_keep(sc, frac=0.65):
    """Shift each asset's output bias so that `frac` of its in-frustum pairs
    have logit >= 0; the threshold is put midway between two neighbouring
    logits so that no pair sits on it."""
    st, lg = oracle.query(sc)
    off = sc.pair_offsets()
    for a_idx, a in enumerate(sc.assets):
        zs = []
        for i, inst in enumerate(sc.instances):
            if inst.asset == a_idx:
                z = lg[:, off[i]:off[i + 1]]
                zs.append(z[~np.isnan(z)])
        z = np.sort(np.concatenate(zs)) if zs else np.zeros(0)
        if len(z) < 2:
            continue
        k = int(np.clip(round((1 - frac) * len(z)), 1, len(z) - 1))
        thr = 0.5 * (z[k - 1] + z[k])
        p = a.mlp.params.copy()
        bo = synth.COMPACT_VIS_PARAMS - 1 if a.mlp.kind == 1 else -1  # the output bias
        p[bo] = np.float32(p[bo] - thr)
        a.mlp.params = p
    return sc


def small_composed(n=6000, n_inst=12, res=(320, 192), seed=77, width=64, degree=3):
    sc = synth.scene_composed(n_per_asset=n, n_inst=n_inst, seed=seed, width=width, res=res, sh_degree=degree,
                              half_extent=6.0)
    sc.cameras = [synth.camera((0.0, -12.0, 5.0), fovy_deg=50.0, width=res[0], height=res[1])]
    return sc


def tiny(n=20000, res=256, width=64):
    return calibrate_keep(synth.scene_tiny(n=n, res=res, width=width))


def composed_small(**kw):
    return calibrate_keep(small_composed(**kw))


def small_batched(frame=0, n_cams=3, res=(160, 96), width=64):
    """The batching workload's recipe at test size: 5 uneven assets, 40
    Zipf-distributed instances, a ring of cameras turned by `frame` degrees."""
    return synth.scene_batched(n_assets=5, n_inst=40, n_cams=n_cams, res=res, n_lo=500, n_hi=4000,
                               half_extent=6.0, frame=frame, ring_radius=8.0, ring_height=2.5, width=width)


def batched_small(**kw):
    return calibrate_keep(small_batched(**kw))


def compact(sc, lo=0.5, hi=1.3, seed=50):
    """The scene with every asset switched to the compact MLP form (Sec. 3.2).
    Each asset's distance range is set from the FoV-corrected camera distances
    of its instances (lo and hi times their median), so that some pairs clamp
    at either end of the range and the nearest segments fall below d_min."""
    d = {}
    for cam in sc.cameras:
        for inst in sc.instances:
            a = sc.assets[inst.asset]
            d.setdefault(inst.asset, []).append(np.linalg.norm(oracle.local_camera(inst, cam, a.mlp.train_focal)))
    for j in range(len(sc.assets)):
        med = float(np.median(d.get(j, [1.0])))
        sc.assets[j] = synth.make_compact(sc.assets[j], seed + j, d_min=lo * med, d_max=hi * med)
    return calibrate_keep(sc)


def tiny_compact(n=20000, res=256):
    return compact(synth.scene_tiny(n=n, res=res, width=64))


def batched_compact(**kw):
    return compact(small_batched(**kw), lo=0.8, hi=2.0)
