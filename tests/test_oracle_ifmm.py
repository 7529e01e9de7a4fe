"""Pins of the oracle's IFMM factorisation and solve.

* eps -> 0: the extended system is equivalent to the matrix it represents
  (eq. ext and Sec. 2.2), so exact elimination must reproduce a dense LU
  solve of that matrix.
* finite eps: the compression is relative, so the normwise backward error
  ||A x - b|| / (||A|| ||x|| + ||b||) of the solve is of order eps.  (The
  residual itself carries a factor cond(A), which reaches 1e5 for i.i.d.
  random points with their near-coincident pairs.)
* symmetry: with unit weights the Laplace matrix, the Chebyshev operators
  and every step of the elimination are symmetric, so the approximate inverse
  must be symmetric to roundoff (catches transposed operands).
* the colour loop: the order inside a colour must not matter (Sec. 3).
"""
import numpy as np
import pytest

import synth
from oracle.ifmm import IFMM, dense_tilde


def _case(shape, N, seed, area):
    pts = synth.geometry_points(shape, N, seed)
    dg = synth.laplace_self_term(N, area)
    return pts, dg


@pytest.mark.parametrize("shape,N,leaf,sigma", [("sphere", 500, 8, 3), ("ellipsoid", 450, 8, 6),
                                                 ("cube", 400, 12, 3)])
def test_exact_limit_matches_dense_lu(shape, N, leaf, sigma):
    area = {"sphere": 4 * np.pi, "ellipsoid": 4 * np.pi * 0.6, "cube": 24.0}[shape]
    pts, dg = _case(shape, N, 21, area)
    b = synth.uniform_rhs(N, 2, 101)
    At = dense_tilde(pts, None, dg, leaf_max=leaf)
    xd = np.linalg.solve(At, b)
    F = IFMM(pts, eps=1e-14, sigma=sigma, diag=dg, leaf_max=leaf).factor()
    assert F.depth >= 3
    x = F.solve(b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10


def test_exact_limit_weighted_columns():
    # non-unit quadrature weights and a per-point diagonal (the BEM form)
    N = 400
    pts = synth.sphere_points(N, 4)
    rng = np.random.default_rng(4)
    w = rng.uniform(0.5, 2.0, N) * (4 * np.pi / N)
    dg = w * synth.laplace_self_term(N) * (N / (4 * np.pi))
    b = synth.uniform_rhs(N, 1, 7)[:, 0]
    At = dense_tilde(pts, w, dg, leaf_max=10)
    F = IFMM(pts, eps=1e-14, sigma=3, diag=dg, weights=w, leaf_max=10).factor()
    x = F.solve(b)
    xd = np.linalg.solve(At, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-10


def test_eps_accuracy_and_monotone():
    N = 1000
    pts, dg = _case("sphere", N, 1, 4 * np.pi)
    b = synth.uniform_rhs(N, 1, 101)[:, 0]
    At = dense_tilde(pts, None, dg, leaf_max=32)
    normA = np.linalg.norm(At, 2)
    res = []
    for eps in (1e-3, 1e-6, 1e-9):
        F = IFMM(pts, eps=eps, sigma=6, diag=dg, leaf_max=32).factor()
        x = F.solve(b)
        r = np.linalg.norm(At @ x - b)
        res.append(r / np.linalg.norm(b))
        bwd = r / (normA * np.linalg.norm(x) + np.linalg.norm(b))
        assert bwd <= 10 * eps
    assert res[0] > res[1] > res[2]


def test_backward_error_ill_conditioned_cube():
    N = 700
    pts, dg = _case("cube", N, 7, 24.0)
    b = synth.uniform_rhs(N, 1, 3)[:, 0]
    At = dense_tilde(pts, None, dg, leaf_max=12)
    eps = 1e-6
    F = IFMM(pts, eps=eps, sigma=3, diag=dg, leaf_max=12).factor()
    x = F.solve(b)
    r = np.linalg.norm(At @ x - b)
    assert r / (np.linalg.norm(At, 2) * np.linalg.norm(x) + np.linalg.norm(b)) <= 10 * eps


@pytest.mark.parametrize("N,leaf", [(800, 32), (1500, 24)])
def test_symmetry_preserved(N, leaf):
    # sizes chosen so that ranks fall below n (real compression of fill-in)
    pts, dg = _case("sphere", N, 9, 4 * np.pi)
    F = IFMM(pts, eps=1e-4, sigma=3, diag=dg, leaf_max=leaf).factor()
    assert any(F.state[l]["r"].sum() < F.state[l]["n"].sum() for l in F.ranks())
    M = F.solve(np.eye(N))
    assert np.linalg.norm(M - M.T) <= 1e-11 * np.linalg.norm(M)


def test_order_inside_colour_is_irrelevant_and_linear():
    N = 500
    pts, dg = _case("ellipsoid", N, 3, 4 * np.pi * 0.6)
    b = synth.uniform_rhs(N, 3, 5)
    F1 = IFMM(pts, eps=1e-6, sigma=3, diag=dg, leaf_max=10).factor()
    rng = np.random.default_rng(0)
    F2 = IFMM(pts, eps=1e-6, sigma=3, diag=dg, leaf_max=10).factor(
        order=lambda lvl, c, nodes: rng.permutation(nodes))
    x1 = F1.solve(b)
    x2 = F2.solve(b)
    assert np.array_equal(x1, x2)
    # multi-RHS equals column-by-column; linearity
    for k in range(3):
        assert np.allclose(F1.solve(b[:, k]), x1[:, k], rtol=0, atol=1e-13 * np.abs(x1).max())
    comb = F1.solve(2.0 * b[:, 0] - 0.5 * b[:, 1])
    assert np.allclose(comb, 2.0 * x1[:, 0] - 0.5 * x1[:, 1], rtol=0, atol=1e-12 * np.abs(x1).max())


def test_rejects_bad_arguments():
    pts = synth.sphere_points(100, 1)
    with pytest.raises(ValueError):
        IFMM(pts, eps=1e-6, sigma=2, diag=1.0)
    with pytest.raises(ValueError):
        IFMM(pts, eps=0.0, sigma=3, diag=1.0)
    with pytest.raises(ValueError):
        IFMM(np.zeros((5, 3)), eps=1e-3, sigma=3, diag=1.0)
    with pytest.raises(RuntimeError):
        IFMM(pts, eps=1e-3, sigma=3, diag=1.0).solve(np.ones(100))
