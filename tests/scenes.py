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
        p[-1] = np.float32(p[-1] - thr)
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
