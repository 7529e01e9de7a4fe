"""Oracle: black-box (Chebyshev) FMM operators for the 3-D Laplace kernel.

Test infrastructure only (see the package header).

Sec. 4.2 of the paper allows the IFMM to be built on a different FMM than the
one used for the matrix-vector product, naming the black-box FMM of Fong and
Darve.  This module writes that FMM's operators out from their definition:

* Chebyshev nodes of the first kind  xb_m = cos((2m - 1) pi / (2 n)), m = 1..n.
* Interpolation weight  S_n(xb, y) = 1/n + (2/n) sum_{k=1}^{n-1} T_k(xb) T_k(y),
  whose value at the node xb_m is the Lagrange basis polynomial of that node;
  in 3-D the weight is the product over the three coordinates.
* P2M_p[m, j] = S(xb_m, y_j) w_j   (y_j: point j in the box's normalised frame)
* L2P_p[j, m] = S(xb_m, y_j)
* M2M_c[m, m'] = S(xb_m, child node m' in the parent's frame); L2L_c = M2M_c^T
* M2L_pl[m, m'] = K(node m of box p, node m' of box l)
* P2P_pq = the matrix A restricted to the points of p and q.

The Laplace kernel is K(x, y) = 1 / (4 pi |x - y|) (the Coulomb example of
Sec. 2, read with the permittivity folded into the scale and the garbled
factor x_i dropped).  Matrix entries are A_ij = K(p_i, p_j) w_j for i != j and
A_ii = diag_i.

3-D node index: m = m1 + n (m2 + n m3) with m1 the x index (fastest).
"""
from __future__ import annotations

import numpy as np

FOUR_PI = 4.0 * np.pi


def cheb_nodes(n: int) -> np.ndarray:
    m = np.arange(1, n + 1, dtype=np.float64)
    return np.cos((2.0 * m - 1.0) * np.pi / (2.0 * n))


def cheb_T(y: np.ndarray, kmax: int) -> np.ndarray:
    """T_0..T_kmax at y (three-term recurrence); shape (kmax + 1, len(y))."""
    y = np.asarray(y, dtype=np.float64)
    T = np.empty((kmax + 1,) + y.shape)
    T[0] = 1.0
    if kmax >= 1:
        T[1] = y
    for k in range(1, kmax):
        T[k + 1] = 2.0 * y * T[k] - T[k - 1]
    return T


def S1(n: int, y: np.ndarray) -> np.ndarray:
    """1-D interpolation weights S_n(xb_m, y): shape (n, len(y))."""
    xb = cheb_nodes(n)
    Tx = cheb_T(xb, n - 1)  # (n, n): Tx[k, m]
    Ty = cheb_T(y, n - 1)   # (n, len(y))
    out = np.full((n, len(y)), 1.0 / n)
    for k in range(1, n):
        out += (2.0 / n) * np.outer(Tx[k], Ty[k])
    return out


def S3(n: int, yhat: np.ndarray) -> np.ndarray:
    """3-D weights: rows = the n^3 Chebyshev nodes, columns = the points yhat (P, 3)."""
    sx = S1(n, yhat[:, 0])
    sy = S1(n, yhat[:, 1])
    sz = S1(n, yhat[:, 2])
    # m = m1 + n*(m2 + n*m3)
    out = sz[:, None, None, :] * sy[None, :, None, :] * sx[None, None, :, :]
    return out.reshape(n ** 3, yhat.shape[0])


_GRID = {}


def node_grid(n: int) -> np.ndarray:
    """The n^3 Chebyshev nodes in the normalised frame, shape (n^3, 3)."""
    if n in _GRID:
        return _GRID[n]
    xb = cheb_nodes(n)
    g = np.empty((n ** 3, 3))
    idx = 0
    for m3 in range(n):
        for m2 in range(n):
            for m1 in range(n):
                g[idx] = (xb[m1], xb[m2], xb[m3])
                idx += 1
    g.setflags(write=False)
    _GRID[n] = g
    return g


def laplace(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """K(x_a, y_b) = 1 / (4 pi |x_a - y_b|) for point sets x (A,3), y (B,3)."""
    d = x[:, None, :] - y[None, :, :]
    r = np.sqrt(np.sum(d * d, axis=2))
    return 1.0 / (FOUR_PI * r)


def p2m(n: int, centre, half, pts, w) -> np.ndarray:
    """P2M of a box: (n^3, P) = S(xb_m, (y_j - c)/h) * w_j."""
    yhat = (pts - centre) / half
    return S3(n, yhat) * w[None, :]


def l2p(n: int, centre, half, pts) -> np.ndarray:
    """L2P of a box: (P, n^3) = S(xb_m, (y_j - c)/h)."""
    yhat = (pts - centre) / half
    return S3(n, yhat).T


def m2m(n: int, octant) -> np.ndarray:
    """M2M from a child in `octant` (each entry -1 or +1 per axis, child centre
    relative to the parent) to its parent: (n^3 parent, n^3 child)."""
    child_nodes = node_grid(n) * 0.5 + 0.5 * np.asarray(octant, dtype=np.float64)[None, :]
    return S3(n, child_nodes)


def m2l(n: int, c_tgt, c_src, half) -> np.ndarray:
    """M2L from source box (centre c_src) to target box (centre c_tgt), both of
    half-side `half`: (n^3 target, n^3 source)."""
    g = node_grid(n)
    return laplace(c_tgt + half * g, c_src + half * g)


def p2p(xt, xs, ws, diag_t=None, same=False) -> np.ndarray:
    """Near-field block A[t, s] = K(x_t, x_s) w_s; on a self block (same=True)
    the diagonal holds diag_t instead of the singular kernel value."""
    if same:
        d = xt[:, None, :] - xs[None, :, :]
        r = np.sqrt(np.sum(d * d, axis=2))
        np.fill_diagonal(r, 1.0)
        B = 1.0 / (FOUR_PI * r) * ws[None, :]
        np.fill_diagonal(B, diag_t)
        return B
    return laplace(xt, xs) * ws[None, :]


def dense_matrix(points, weights, diag) -> np.ndarray:
    """The full N x N matrix A (tiny N only)."""
    n = points.shape[0]
    A = p2p(points, points, weights, diag_t=diag, same=True)
    assert A.shape == (n, n)
    return A
