"""Writes the oracle's solutions of the N = 65,536 sphere workload (seed 2,
Laplace kernel, leaves of at most 64 points, Chebyshev 4^3, eps = 1e-6,
8 right-hand sides U[-1, 1] with seeds 201..208, one seed per column) for
sigma = 3 and sigma = 6, with the oracle's ranks per level.

Only the CPU oracle (oracle/) and the seeded generators (synth/) run here.
Output: cfg2_sphere65536_sigma{3,6}.npz beside this script.
Run: python tests/golden/make_cfg2.py  (about 10 minutes per sigma on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle.ifmm import IFMM  # noqa: E402

N, SEED, EPS, LEAF = 65536, 2, 1e-6, 64
RHS_SEEDS = list(range(201, 209))


def inputs():
    pts = synth.sphere_points(N, SEED)
    dg = synth.laplace_self_term(N)
    b = np.asfortranarray(np.concatenate([synth.uniform_rhs(N, 1, s) for s in RHS_SEEDS], axis=1))
    return pts, dg, b


def main(sigmas=(3, 6)):
    pts, dg, b = inputs()
    for sigma in sigmas:
        t0 = time.time()
        F = IFMM(pts, eps=EPS, sigma=sigma, diag=dg, leaf_max=LEAF).factor()
        x = F.solve(b)
        ranks = {f"ranks_level{l}": np.asarray(F.state[l]["r"], dtype=np.int32) for l in range(2, F.depth + 1)}
        out = os.path.join(HERE, f"cfg2_sphere65536_sigma{sigma}.npz")
        np.savez_compressed(out, x=x, depth=np.int32(F.depth), eps=EPS, sigma=np.int32(sigma), **ranks)
        print(f"sigma={sigma}: depth {F.depth}, oracle factor+solve {time.time() - t0:.1f} s -> {out}", flush=True)


if __name__ == "__main__":
    main(tuple(int(a) for a in sys.argv[1:]) or (3, 6))
