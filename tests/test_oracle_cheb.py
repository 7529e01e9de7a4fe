"""Pins of the oracle's Chebyshev (black-box FMM) operators."""
import numpy as np
import pytest

import synth
from oracle import cheb
from oracle.ifmm import dense_tilde


@pytest.mark.parametrize("n", [3, 4, 5])
def test_interpolation_reproduces_polynomials(n):
    # S_n(xb_m, .) are the Lagrange polynomials of the Chebyshev nodes:
    # sum_m f(xb_m) S_n(xb_m, y) == f(y) for every f of degree < n.
    rng = np.random.default_rng(n)
    y = rng.uniform(-1, 1, size=(50, 3))
    g = cheb.node_grid(n)
    coef = rng.standard_normal((n, n, n))

    def f(p):
        out = 0.0
        for a in range(n):
            for b in range(n):
                for c in range(n):
                    out = out + coef[a, b, c] * p[..., 0] ** a * p[..., 1] ** b * p[..., 2] ** c
        return out

    approx = f(g) @ cheb.S3(n, y)
    assert np.allclose(approx, f(y), rtol=0, atol=1e-11 * np.abs(f(y)).max())
    # partition of unity
    assert np.allclose(cheb.S3(n, y).sum(axis=0), 1.0, atol=1e-13)
    # nodal property
    assert np.allclose(cheb.S3(n, g), np.eye(n ** 3), atol=1e-13)


def test_m2m_p2m_consistency():
    # M2M_c P2M_c = P2M_parent on the child's points (exact polynomial reproduction)
    rng = np.random.default_rng(1)
    n = 4
    cp, hp = np.array([0.3, -0.2, 0.1]), 0.5
    for octant in [(-1, -1, -1), (1, -1, 1), (1, 1, 1)]:
        o = np.array(octant, float)
        cc, hc = cp + 0.5 * hp * o, 0.5 * hp
        pts = cc + hc * rng.uniform(-1, 1, size=(20, 3))
        w = rng.uniform(0.5, 2.0, size=20)
        lhs = cheb.m2m(n, o) @ cheb.p2m(n, cc, hc, pts, w)
        rhs = cheb.p2m(n, cp, hp, pts, w)
        assert np.allclose(lhs, rhs, atol=1e-13)
        # L2L = M2M^T is the matching local translation
        lhs = cheb.l2p(n, cc, hc, pts) @ cheb.m2m(n, o).T
        assert np.allclose(lhs, cheb.l2p(n, cp, hp, pts), atol=1e-13)


def test_far_field_converges_with_order():
    # L2P M2L P2M approximates the kernel between well-separated boxes, with
    # an error that falls as the Chebyshev order grows.
    rng = np.random.default_rng(2)
    h = 0.5
    ct, cs = np.zeros(3), np.array([2.0, 1.0, 0.0]) * (2 * h)
    xt = ct + h * rng.uniform(-1, 1, (30, 3))
    xs = cs + h * rng.uniform(-1, 1, (30, 3))
    w = np.ones(30)
    exact = cheb.laplace(xt, xs)
    errs = []
    for n in (2, 3, 4, 5, 6):
        approx = cheb.l2p(n, ct, h, xt) @ cheb.m2l(n, ct, cs, h) @ cheb.p2m(n, cs, h, xs, w)
        errs.append(np.abs(approx - exact).max() / np.abs(exact).max())
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[2] < 5e-3


def test_dense_tilde_close_to_A():
    N = 400
    pts = synth.sphere_points(N, 5)
    dg = synth.laplace_self_term(N)
    A = cheb.dense_matrix(pts, np.ones(N), np.full(N, dg))
    At = dense_tilde(pts, None, dg, leaf_max=8)
    rel = np.linalg.norm(At - A) / np.linalg.norm(A)
    assert 0 < rel < 1e-2
    # near blocks are exact copies of A
    from oracle.tree import Tree, dist
    T = Tree(pts, leaf_max=8)
    leaf = T.levels[T.depth]
    for p in range(0, leaf.n, 7):
        for q in leaf.nbr[p] + [p]:
            ip, iq = T.leaf_points(p), T.leaf_points(q)
            assert np.array_equal(At[np.ix_(ip, iq)], A[np.ix_(ip, iq)])
