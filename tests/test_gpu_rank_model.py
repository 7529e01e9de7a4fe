"""The learned recompression rank: device network against the FP64 oracle
(oracle/mlp.py), training on the device, and the factorisation with the
trained model against the FP64 oracle of the IFMM.

Tolerances: the device network runs in FP32, so forward values and
gradients agree with the FP64 oracle to ~1e-5 relative (1e-4 asserted); a
short training run follows the oracle's Adam trajectory to 1e-3 relative in
the loss.  The factorisation with the model keeps the accuracy bar of the
plain path (10 eps against the oracle), since every sketch passes the
a-posteriori test or falls back to the full decomposition.
"""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from oracle.ifmm import IFMM as Oracle

pytestmark = pytest.mark.gpu
F = 14


def _data(m, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, F)).astype(np.float32)
    t = (0.3 + 0.2 * np.tanh(X[:, 0]) + 0.05 * X[:, 1] ** 2).astype(np.float32)
    return X, t


def test_forward_and_gradient_match_oracle():
    from paper_1905_10602_amd import rank_model_eval, rank_model_grad, rank_model_params
    assert rank_model_params(F) == omlp.n_params(F)
    X, t = _data(300, 1)
    th = omlp.init(F, 2).astype(np.float32)
    y = rank_model_eval(th, X)
    yo, _ = omlp.forward(th.astype(np.float64), X.astype(np.float64), F)
    assert np.allclose(y, yo, rtol=1e-4, atol=1e-5 * np.abs(yo).max())
    for tau in (0.5, 0.9):
        L, g = rank_model_grad(th, X, t, tau)
        Lo, go = omlp.loss_and_grad(th.astype(np.float64), X.astype(np.float64), t.astype(np.float64), F, tau)
        assert abs(L - Lo) <= 1e-4 * abs(Lo)
        assert np.allclose(g, go, rtol=1e-3, atol=1e-4 * np.abs(go).max())


def test_training_follows_oracle_adam():
    from paper_1905_10602_amd import rank_model_train
    X, t = _data(400, 3)
    th0 = omlp.init(F, 4)
    th, hist = rank_model_train(X, t, th0.astype(np.float32), 20, lr=1e-3, tau=0.9)
    tho = th0.copy()
    m1 = np.zeros_like(tho)
    m2 = np.zeros_like(tho)
    ho = []
    for k in range(1, 21):
        L, g = omlp.loss_and_grad(tho, X.astype(np.float64), t.astype(np.float64), F, 0.9)
        ho.append(L)
        tho, m1, m2 = omlp.adam_step(tho, g, m1, m2, k, 1e-3)
    assert np.allclose(hist, ho, rtol=1e-3)
    assert np.allclose(th, tho, rtol=0, atol=2e-4 * np.abs(tho).max())
    # longer run: the loss falls
    th2, hist2 = rank_model_train(X, t, th0.astype(np.float32), 500, lr=2e-3, tau=0.9)
    assert hist2[-1] < 0.5 * hist2[0]


def test_learned_rank_factorisation():
    from paper_1905_10602_amd import IFMM, rank_model_train
    from paper_1905_10602_amd.rank_model import init_params
    eps = 1e-6
    # training records from geometries other than the test one
    Xs, ts = [], []
    for seed, shape in ((11, "ellipsoid"), (12, "sphere"), (13, "ellipsoid")):
        kw = {"jitter": 0.05} if shape == "ellipsoid" else {}
        pts = synth.geometry_points(shape, 12000, seed, **kw)
        h = IFMM(pts, eps, 3, diag=synth.laplace_self_term(12000), leaf_max=32)
        h.record_ranks(True)
        h.factor()
        X, t = h.rank_records()
        assert X.shape == (len(t), F) and len(t) > 50
        assert np.all((t >= 0) & (t <= 1)) and np.all(np.isfinite(X))
        Xs.append(X)
        ts.append(t)
    X, t = np.concatenate(Xs), np.concatenate(ts)
    th, hist = rank_model_train(X, t, init_params(0), 1500, lr=2e-3, tau=0.9)
    assert hist[-1] < hist[0]
    # test geometry, small enough for the oracle
    N = 4096
    pts = synth.ellipsoid_points(N, 21, jitter=0.05)
    dg = synth.laplace_self_term(N, 2.6)
    b = synth.uniform_rhs(N, 2, 5)
    xo = Oracle(pts, eps=eps, sigma=3, diag=dg, leaf_max=32).factor().solve(b)
    hm = IFMM(pts, eps, 3, diag=dg, leaf_max=32).set_rank_model(th).factor()
    st = hm.stats()
    print(f"learned: predictions {st['rank_predictions']} sketches {st['sketches']} "
          f"rejected {st['sketches_rejected']}", flush=True)
    assert st["rank_predictions"] > 0
    x = hm.solve(b)
    assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 10 * eps
    # what the network gains over the method without it: full decompositions avoided
    h0 = IFMM(pts, eps, 3, diag=dg, leaf_max=32).factor()
    s0 = h0.stats()
    full_with = st["changed"] - (st["sketches"] - st["sketches_rejected"])
    print(f"full eigen-decompositions: {st['changed']} without sketches, {full_with} with the model; "
          f"heuristic sketch: {s0['sketches']} tried, {s0['sketches_rejected']} rejected", flush=True)
    assert st["sketches"] - st["sketches_rejected"] > 0


def test_trained_model_against_rule_on_held_out_geometry():
    # What the committed network gains over the rule without it, on a geometry
    # outside its training set (ellipsoid, seed 6001, N = 131,072, eps 1e-6,
    # sigma 3, cost-model bottom level): every sketch-eligible recompression is
    # recorded with the rank the full truncation chose.  A sketch of width s
    # can only be accepted when that rank is below s.  Compared: the model's
    # widths (prediction + max(8, pred / 8)) and the rule's (current rank +
    # max(16, r / 4)).  On its training geometries the model misses the rank
    # about ten times less often than the rule at the same mean width; on this
    # held-out geometry the two are about even (4.5 % against 4.2 % misses,
    # mean widths 85.0 and 85.7), so the test asserts only that the model is
    # no worse than the rule by more than a small margin, and prints both.
    # The factor time at N = 1M is reported by the benchmark (the
    # learned_rank_ablation entry), not asserted here.
    from paper_1905_10602_amd import IFMM, rank_model_eval
    from paper_1905_10602_amd.rank_model import load
    theta, meta = load()
    N, eps = 131072, 1e-6
    print(f"case trained model vs rule: ellipsoid seed 6001 N={N}", flush=True)
    axes = (1.0, 0.6, 0.4)
    pts = synth.ellipsoid_points(N, 6001, axes=axes, jitter=0.05)
    h = IFMM(pts, eps, 3, diag=synth.laplace_self_term(N, synth.ellipsoid_area(axes)), leaf_max=64,
             bottom_level=-1)
    h.record_ranks(True)
    h.factor()
    X, t = h.rank_records()
    h.close()
    assert len(t) > 1000
    n = np.rint(X[:, 4] * 1024).astype(np.int64)
    r = np.rint(X[:, 5] * 512).astype(np.int64)
    rnew = np.rint(t * n).astype(np.int64)
    fr = np.clip(rank_model_eval(theta, X), 0.0, 1.0)
    pred = np.maximum(1, np.ceil(fr * n)).astype(np.int64)
    s_model = np.minimum(n, pred + np.maximum(8, pred // 8))
    s_rule = np.minimum(n, r + np.maximum(16, r // 4))
    both = (s_model <= 0.6 * n) & (s_rule <= 0.6 * n)
    miss_model = float(np.mean(rnew[both] >= s_model[both]))
    miss_rule = float(np.mean(rnew[both] >= s_rule[both]))
    w_model, w_rule = float(np.mean(s_model[both])), float(np.mean(s_rule[both]))
    print(f"{int(both.sum())} recompressions: rank above the width {miss_model:.4f} (model) vs {miss_rule:.4f} "
          f"(rule); mean width {w_model:.1f} vs {w_rule:.1f}; model trained on {meta['samples']} samples", flush=True)
    assert miss_model <= 1.5 * miss_rule + 0.01
    assert w_model <= 1.1 * w_rule
