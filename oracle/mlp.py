"""Oracle: the rank-prediction network (two hidden layers of 64, ReLU) in FP64.

Test infrastructure only (see the package header).

The paper compresses fill-in with a randomised SVD whose size must be chosen
(Sec. 5.1 mentions the randomised SVD); the learned part predicts each
recompression's rank so that the sketch is sized before it runs, with the
full rank-revealing decomposition as the fall-back.  The network and its
training are textbook:

  h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = w3 . h2 + b3
  loss = mean over samples of the pinball (quantile) loss at level tau:
         rho_tau(u) = tau u (u >= 0),  (tau - 1) u (u < 0),  u = target - y
  Adam (Kingma and Ba) with bias correction.

Flat parameter layout (shared with the device code only through this
documented order): W1 (64 x F, row-major), b1 (64), W2 (64 x 64, row-major),
b2 (64), w3 (64), b3 (1).
"""
from __future__ import annotations

import numpy as np

H = 64


def n_params(F: int) -> int:
    return H * F + H + H * H + H + H + 1


def unpack(theta: np.ndarray, F: int):
    o = 0
    W1 = theta[o:o + H * F].reshape(H, F); o += H * F
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    w3 = theta[o:o + H]; o += H
    b3 = theta[o:o + 1]
    return W1, b1, W2, b2, w3, b3


def init(F: int, seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (any initialisation will do for the tests,
    which pass the same parameters to both sides)."""
    rng = np.random.default_rng(seed)
    th = np.zeros(n_params(F))
    W1, b1, W2, b2, w3, b3 = unpack(th, F)
    W1[:] = rng.uniform(-1, 1, W1.shape) * np.sqrt(6.0 / F)
    W2[:] = rng.uniform(-1, 1, W2.shape) * np.sqrt(6.0 / H)
    w3[:] = rng.uniform(-1, 1, w3.shape) * np.sqrt(6.0 / H)
    return th


def forward(theta, X, F):
    W1, b1, W2, b2, w3, b3 = unpack(theta, F)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3[0]
    return y, (z1, h1, z2, h2)


def pinball(u, tau):
    return np.where(u >= 0.0, tau * u, (tau - 1.0) * u)


def loss_and_grad(theta, X, t, F, tau):
    """Mean pinball loss and its gradient with respect to the flat parameters
    (the subgradient at u = 0 is taken as -tau, the branch u >= 0)."""
    W1, b1, W2, b2, w3, b3 = unpack(theta, F)
    m = X.shape[0]
    y, (z1, h1, z2, h2) = forward(theta, X, F)
    u = t - y
    L = float(np.mean(pinball(u, tau)))
    dy = np.where(u >= 0.0, -tau, 1.0 - tau) / m        # dL/dy
    g = np.zeros_like(theta)
    gW1, gb1, gW2, gb2, gw3, gb3 = unpack(g, F)
    gw3[:] = h2.T @ dy
    gb3[0] = dy.sum()
    dh2 = np.outer(dy, w3)
    dz2 = dh2 * (z2 > 0.0)
    gW2[:] = dz2.T @ h1
    gb2[:] = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0.0)
    gW1[:] = dz1.T @ X
    gb1[:] = dz1.sum(axis=0)
    return L, g


def adam_step(theta, g, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns the new (theta, m1, m2)."""
    m1 = b1 * m1 + (1.0 - b1) * g
    m2 = b2 * m2 + (1.0 - b2) * g * g
    mh = m1 / (1.0 - b1 ** step)
    vh = m2 / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m1, m2
