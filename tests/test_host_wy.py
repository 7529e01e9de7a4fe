"""The compact WY form that the blocked eigenvector back-transform applies.

For unit Householder vectors v_q (zero on and above row q, H_q = I - 2 v_q
v_q^T; a skipped reflector has v_q = 0 and H_q = I) the product
H_b0 ... H_b1-1 equals I - V T V^T with T^-1 = diag(1/2) + (strict upper part
of V^T V) (Joffrain, Low, Quintana-Orti, van de Geijn and Van Zee,
"Accumulating Householder transformations, revisited", 2006).  The kernel
forms W = T (V^T X) by back substitution with T^-1 and updates X -= V W; both
are checked here against the explicit product of the reflectors.
"""
import numpy as np
import pytest


def _reflectors(n, b0, nb, rng, skip=()):
    V = np.zeros((n, nb))
    for c in range(nb):
        q = b0 + c
        if c in skip:
            continue
        x = rng.standard_normal(n - q - 1)
        V[q + 1:, c] = x / np.linalg.norm(x)
    return V


@pytest.mark.parametrize("n,b0,nb,skip", [(40, 0, 32, ()), (70, 5, 32, (3, 17)), (50, 20, 28, (0,)), (9, 0, 7, ())])
def test_compact_wy_equals_the_product_of_reflectors(n, b0, nb, skip):
    rng = np.random.default_rng(1000 * n + b0)
    V = _reflectors(n, b0, nb, rng, skip)
    H = np.eye(n)
    for c in range(nb):
        H = H @ (np.eye(n) - 2.0 * np.outer(V[:, c], V[:, c]))
    G = V.T @ V
    t_inv = np.diag(np.full(nb, 0.5)) + np.triu(G, 1)
    assert np.allclose(np.eye(n) - V @ np.linalg.inv(t_inv) @ V.T, H, atol=1e-12)
    # the kernel's steps on a block of columns: B = V^T X, back substitution
    # W[q] = 2 (B[q] - sum_{p > q} G[q, p] W[p]), then X - V W
    X = rng.standard_normal((n, 5))
    B = V.T @ X
    W = np.zeros_like(B)
    for q in range(nb - 1, -1, -1):
        W[q] = 2.0 * (B[q] - G[q, q + 1:] @ W[q + 1:])
    assert np.allclose(X - V @ W, H @ X, atol=1e-12)


def test_a_wrong_diagonal_is_caught():
    # the identity needs the 1/2 of the unit-vector reflectors (tau = 2): with
    # diag 1 instead the product is not reproduced
    rng = np.random.default_rng(7)
    n, nb = 30, 8
    V = _reflectors(n, 0, nb, rng)
    H = np.eye(n)
    for c in range(nb):
        H = H @ (np.eye(n) - 2.0 * np.outer(V[:, c], V[:, c]))
    t_bad = np.eye(nb) + np.triu(V.T @ V, 1)
    assert not np.allclose(np.eye(n) - V @ np.linalg.inv(t_bad) @ V.T, H, atol=1e-6)
