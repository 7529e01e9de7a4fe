"""Pins of the FMM, FGMRES and BEM oracles against definitions that do not use them.

* FMM: the hierarchical passes must reproduce, up to rounding, the matrix
  A~ that ``dense_tilde`` forms block by block from the same Chebyshev
  operators (a different construction), and approach the dense matrix A as
  the Chebyshev order grows (interpolation error).
* FGMRES: finite termination on an n x n system with restart >= n, the exact
  inverse as preconditioner converging in one step, the returned residual
  estimate equal to the true residual (which a wrong Givens sign or a
  dropped Hessenberg entry breaks).
* BEM: the discrete density converges to the closed-form sigma of a point
  source inside the unit sphere.
"""
import numpy as np
import pytest

from oracle import bem, cheb
from oracle.fmm import FMM
from oracle.ifmm import dense_tilde
from oracle.krylov import fgmres, givens
from synth import icosphere, sphere_points, uniform_rhs


@pytest.mark.parametrize("n,leaf,nc", [(700, 32, 5), (900, 24, 4)])
def test_fmm_equals_dense_tilde(n, leaf, nc):
    pts = sphere_points(n, 11)
    w = np.random.default_rng(3).uniform(0.5, 1.5, n)
    x = uniform_rhs(n, 2, 12)
    F = FMM(pts, w, 1.7, leaf_max=leaf, cheb_order=nc)
    At = dense_tilde(pts, w, 1.7, leaf_max=leaf, cheb_order=nc)
    y = F.matvec(x)
    assert np.linalg.norm(y - At @ x) <= 1e-13 * np.linalg.norm(y)
    assert np.allclose(F.matvec(x[:, 0]), y[:, 0], rtol=0, atol=1e-14 * np.abs(y).max())


def test_fmm_interpolation_error_decreases_with_order():
    n = 1000
    pts = sphere_points(n, 4)
    x = uniform_rhs(n, 1, 5)[:, 0]
    A = cheb.dense_matrix(pts, np.ones(n), np.full(n, 2.0))
    y = A @ x
    errs = [np.linalg.norm(FMM(pts, None, 2.0, leaf_max=32, cheb_order=k).matvec(x) - y) / np.linalg.norm(y)
            for k in (3, 4, 5)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-4


def _system(n, seed, shift=4.0):
    rng = np.random.default_rng(seed)
    B = shift * np.eye(n) + rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    return B, b


def test_fgmres_finite_termination():
    B, b = _system(30, 1)
    x, its, rr = fgmres(lambda v: B @ v, b, tol=1e-13, restart=40)
    assert its <= 30
    assert np.linalg.norm(x - np.linalg.solve(B, b)) <= 1e-11 * np.linalg.norm(x)


def test_fgmres_exact_preconditioner_one_step():
    B, b = _system(25, 2)
    Bi = np.linalg.inv(B)
    x, its, rr = fgmres(lambda v: B @ v, b, precond=lambda v: Bi @ v, tol=1e-12)
    assert its == 1
    assert np.linalg.norm(B @ x - b) <= 1e-12 * np.linalg.norm(b)


def test_fgmres_residual_estimate_is_true_residual():
    B, b = _system(60, 3, shift=12.0)  # spectrum away from 0: restarted GMRES converges
    for restart in (60, 10):
        x, its, rr = fgmres(lambda v: B @ v, b, tol=1e-6, restart=restart, maxit=600)
        true = np.linalg.norm(B @ x - b) / np.linalg.norm(b)
        assert rr <= 1e-6
        assert abs(true - rr) <= 1e-9


def test_fgmres_zero_rhs_and_variable_preconditioner():
    B, b = _system(20, 4)
    x, its, rr = fgmres(lambda v: B @ v, np.zeros(20))
    assert its == 0 and not np.any(x)
    # a preconditioner that changes between calls (FGMRES keeps z_j)
    calls = [0]
    D = np.diag(1.0 / np.diag(B))

    def prec(v):
        calls[0] += 1
        return D @ v * (1.0 + 0.1 * (calls[0] % 3))

    x, its, rr = fgmres(lambda v: B @ v, b, precond=prec, tol=1e-10, restart=30, maxit=200)
    assert np.linalg.norm(B @ x - b) <= 1e-9 * np.linalg.norm(b)


def test_givens_zeroes_second_component():
    for a, b in [(3.0, 4.0), (-2.0, 1e-3), (0.0, 5.0), (1.0, 0.0), (-1.0, 0.0)]:
        c, s = givens(a, b)
        assert abs(-s * a + c * b) <= 1e-15 * (abs(a) + abs(b))
        assert c * a + s * b >= 0.0
        assert abs(c * c + s * s - 1.0) <= 1e-15


def test_bem_density_converges_to_closed_form():
    errs = []
    for sd in (2, 3, 4):
        V, T = icosphere(sd)
        c, a = bem.panels(V, T)
        A = bem.dense_matrix(c, a)
        s = np.linalg.solve(A, bem.point_source(c))
        ex = bem.exact_density(c)
        errs.append(np.linalg.norm(s - ex) / np.linalg.norm(ex))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.015


def test_bem_pieces():
    V, T = icosphere(3)
    c, a = bem.panels(V, T)
    assert len(a) == 1280
    assert abs(a.sum() - 4 * np.pi) < 0.02 * 4 * np.pi  # flat panels: slightly less than the sphere
    # self term of a disc equals the centre value of its single-layer potential
    assert np.allclose(bem.self_terms(np.array([np.pi])), 0.5)
    # the closed form reduces to the uniform density 1 for x0 = 0 (f = 1 on the sphere)
    assert np.allclose(bem.exact_density(c / np.linalg.norm(c, axis=1)[:, None], (0.0, 0.0, 0.0)), 1.0)


def test_bd_oracle_inverts_the_block_diagonal_part():
    # BD is exact on the block-diagonal part of A: BD (A_bd x) = x at every
    # level.  On the BEM system (panel areas as weights) wider blocks (coarser
    # l_BD) take no more FGMRES iterations (Sec. 4.3); for this first-kind
    # Laplace operator the leaf BD is no better than no preconditioner
    import synth
    from oracle.bd import BD
    from oracle.bem import dense_matrix, panels, point_source, self_terms
    from oracle.krylov import fgmres
    from oracle.tree import Tree
    v, f = synth.icosphere(4)
    c, a = panels(v, f)
    N = c.shape[0]
    A = dense_matrix(c, a)
    st = self_terms(a)
    x = np.random.default_rng(0).standard_normal(N)
    depth = Tree(c, leaf_max=16, sigma=3).depth
    its = []
    for level in range(depth, 1, -1):
        bd = BD(c, st, weights=a, level=level, leaf_max=16)
        Abd = np.zeros_like(A)
        for idx, _ in bd.boxes:
            Abd[np.ix_(idx, idx)] = A[np.ix_(idx, idx)]
        assert np.allclose(bd.apply(Abd @ x), x, rtol=0, atol=1e-9 * np.abs(x).max())
        _, it, rr = fgmres(lambda y: A @ y, point_source(c), precond=bd.apply, tol=1e-8, restart=50)
        assert rr <= 1e-8
        its.append(it)
    print(f"FGMRES iterations with BD at levels {depth}..2: {its}")
    assert all(b <= a for a, b in zip(its, its[1:]))
