"""Training data and training of the recompression-rank network.

The samples are the library's own recompressions: a factorisation with
``record_ranks`` on stores, for every sketch-eligible changed node, the
features (see include/ifmm.h) and the rank the full truncation rule chose
(as a fraction of n).  Training runs on the device (ifmm_rank_model_train).
The geometries used here are drawn from seeds and shapes disjoint from the
benchmark's workload (an ellipsoid with seed 5).

    python -m paper_1905_10602_amd.rank_model --out paper_1905_10602_amd/rank_model_laplace.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from .ifmm import IFMM, RANK_FEATURES, rank_model_params, rank_model_train

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT = os.path.join(HERE, "rank_model_laplace.npz")


def training_geometries(count=16, n_values=(65536, 131072, 262144), base_seed=5001, large=(524288, 524288, 1048576)):
    """(name, points, diag) of the training set: spheres, ellipsoids with random
    semi-axes in [0.5, 2] (plus 5 % jitter) and cube surfaces, seeds from 5001;
    `count` geometries with N from n_values, then one per entry of `large`
    (the upper levels of large problems carry the largest recompressions)."""
    sys.path.insert(0, os.path.dirname(HERE))
    import synth
    out = []
    sizes = [int(n_values[g % len(n_values)]) for g in range(count)] + [int(v) for v in large]
    for g, n in enumerate(sizes):
        seed = base_seed + g
        rng = np.random.default_rng(seed)
        kind = ("ellipsoid", "sphere", "cube")[g % 3]
        if kind == "ellipsoid":
            axes = tuple(rng.uniform(0.5, 2.0, 3))
            pts = synth.ellipsoid_points(n, seed, axes=axes, jitter=0.05)
            area = synth.ellipsoid_area(axes)
        elif kind == "sphere":
            pts = synth.sphere_points(n, seed)
            area = 4 * np.pi
        else:
            pts = synth.cube_surface_points(n, seed)
            area = 24.0
        out.append((f"{kind}-{n}-{seed}", pts, synth.laplace_self_term(n, area)))
    return out


def record(geoms, eps=1e-6, sigma=3, leaf_max=64, bottom_level=-1, log=print):
    """Samples of every geometry, factorised as the benchmark factorises (the
    cost model's bottom level by default)."""
    Xs, ts = [], []
    for name, pts, dg in geoms:
        t0 = time.time()
        h = IFMM(pts, eps, sigma, diag=dg, leaf_max=leaf_max, bottom_level=bottom_level)
        h.record_ranks(True)
        h.factor()
        X, t = h.rank_records()
        h.close()
        log(f"[rank_model] {name}: {len(t)} samples in {time.time() - t0:.1f} s")
        Xs.append(X)
        ts.append(t)
    return np.concatenate(Xs), np.concatenate(ts)


def init_params(seed=0):
    """He-uniform initial parameters in the documented flat order."""
    F, H = RANK_FEATURES, 64
    rng = np.random.default_rng(seed)
    th = np.zeros(rank_model_params(F), dtype=np.float32)
    o = 0
    th[o:o + H * F] = rng.uniform(-1, 1, H * F) * np.sqrt(6.0 / F); o += H * F + H
    th[o:o + H * H] = rng.uniform(-1, 1, H * H) * np.sqrt(6.0 / H); o += H * H + H
    th[o:o + H] = rng.uniform(-1, 1, H) * np.sqrt(6.0 / H)
    return th


def train(X, t, steps=3000, lr=2e-3, tau=0.9, seed=0):
    th, hist = rank_model_train(X, t, init_params(seed), steps, lr=lr, tau=tau)
    return th, hist


def save(path, theta, meta):
    np.savez(path, theta=theta.astype(np.float32), meta=json.dumps(meta))


def load(path=DEFAULT):
    with np.load(path, allow_pickle=False) as z:
        return z["theta"].astype(np.float32), json.loads(str(z["meta"]))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT)
    ap.add_argument("--count", type=int, default=16)
    ap.add_argument("--records", default=None, help="also save the recorded samples (npz) here")
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--tau", type=float, default=0.9)
    a = ap.parse_args(argv)
    X, t = record(training_geometries(a.count), log=lambda s: print(s, flush=True))
    if a.records:
        np.savez_compressed(a.records, X=X, t=t)
    th, hist = train(X, t, steps=a.steps, tau=a.tau)
    meta = {"samples": int(len(t)), "steps": a.steps, "tau": a.tau, "loss_first": float(hist[0]),
            "loss_last": float(hist[-1]), "features": RANK_FEATURES, "geometries": a.count,
            "seeds": f"5001-{5000 + a.count + 3}", "n_values": [65536, 131072, 262144],
            "large": [524288, 524288, 1048576], "bottom_level": "cost model"}
    save(a.out, th, meta)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
