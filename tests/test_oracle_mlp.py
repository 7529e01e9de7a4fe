"""Pins of the rank-network oracle: gradients against central finite
differences of the loss (which a wrong ReLU mask, a transposed weight or a
missing 1/m breaks), the pinball loss against its quantile property, and
Adam's first step against its closed form (a step of lr * sign(g))."""
import numpy as np

from oracle import mlp


def _data(m, F, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, F))
    t = np.tanh(X[:, 0]) + 0.5 * X[:, 1] ** 2 - 0.3 * X[:, 2]
    return X, t


def test_gradient_matches_finite_differences():
    F = 6
    X, t = _data(40, F, 1)
    th = mlp.init(F, 2)
    th[mlp.H * F: mlp.H * F + mlp.H] = 0.05  # non-zero biases
    for tau in (0.5, 0.9):
        L, g = mlp.loss_and_grad(th, X, t, F, tau)
        rng = np.random.default_rng(3)
        idx = rng.choice(th.size, 60, replace=False)
        h = 1e-6
        for i in idx:
            e = np.zeros_like(th)
            e[i] = h
            Lp, _ = mlp.loss_and_grad(th + e, X, t, F, tau)
            Lm, _ = mlp.loss_and_grad(th - e, X, t, F, tau)
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_pinball_minimiser_is_the_quantile():
    rng = np.random.default_rng(4)
    u = rng.standard_normal(20001)
    grid = np.linspace(-2, 2, 4001)
    for tau in (0.5, 0.9):
        losses = [np.mean(mlp.pinball(u - c, tau)) for c in grid]
        c = grid[int(np.argmin(losses))]
        assert abs(c - np.quantile(u, tau)) < 0.01


def test_adam_first_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th = np.ones(4)
    th1, m1, m2 = mlp.adam_step(th, g, np.zeros(4), np.zeros(4), 1, 0.01)
    expect = th - 0.01 * g / (np.abs(g) + 1e-8)
    assert np.allclose(th1, expect, rtol=0, atol=1e-12)


def test_training_reduces_loss():
    F = 6
    X, t = _data(256, F, 5)
    th = mlp.init(F, 6)
    m1 = np.zeros_like(th)
    m2 = np.zeros_like(th)
    L0, _ = mlp.loss_and_grad(th, X, t, F, 0.5)
    for k in range(1, 301):
        L, g = mlp.loss_and_grad(th, X, t, F, 0.5)
        th, m1, m2 = mlp.adam_step(th, g, m1, m2, k, 3e-3)
    L1, _ = mlp.loss_and_grad(th, X, t, F, 0.5)
    assert L1 < 0.3 * L0
