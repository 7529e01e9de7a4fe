"""Oracle: the black-box (Chebyshev) FMM matrix-vector product.

Test infrastructure only (see the package header).

Sec. 4.1 / Alg. 4 of the paper wrap the IFMM preconditioner around an FMM
matrix-vector product, whose operators are P2M, M2M, M2L, L2L, L2P and P2P
(Alg. 4, precomputation step); Sec. 4.2 allows that FMM to differ from the
one the IFMM is built from and names the black-box FMM of Fong and Darve.
This module evaluates y = A~ x with the operators of ``oracle.cheb`` on the
uniform octree of ``oracle.tree``, in the textbook order:

  upward    m_leaf = P2M x_leaf;  m_parent = sum_children M2M_c m_child
  transfer  l_i = sum_{s in I_i} M2L_is m_s             (every level >= 2)
  downward  l_child += L2L_c l_parent
  leaves    y_leaf = L2P l_leaf + sum_{q in N_i + {i}} P2P_iq x_q

Reading: the FMM uses the same uniform octree (root cube, depth rule) as the
IFMM; the paper's FMM is adaptive but shares the root (Sec. 4.2).  A~ is
then exactly the matrix ``oracle.ifmm.dense_tilde`` forms entry by entry,
with the same Chebyshev order.
"""
from __future__ import annotations

import numpy as np

from . import cheb
from .tree import Tree


def _octant(coord) -> np.ndarray:
    return np.where((np.asarray(coord) & 1) == 1, 1.0, -1.0)


class FMM:
    """Matrix-vector products with A~ for one point set.

    A_ij = K(p_i, p_j) w_j for i != j, A_ii = diag_i, K = 1 / (4 pi r).
    """

    def __init__(self, points, weights=None, diag=0.0, leaf_max=64, cheb_order=5, sigma=6):
        self.points = np.asarray(points, dtype=np.float64)
        N = self.points.shape[0]
        self.w = np.ones(N) if weights is None else np.asarray(weights, dtype=np.float64)
        self.diag = np.full(N, float(diag)) if np.isscalar(diag) else np.asarray(diag, dtype=np.float64)
        self.nc = cheb_order
        self.tree = Tree(self.points, leaf_max=leaf_max, sigma=sigma)
        T = self.tree
        L = T.depth
        leaf = T.levels[L]
        self.p2m = []
        self.l2p = []
        for i in range(leaf.n):
            ip = T.leaf_points(i)
            c, h = T.box(L, i)
            self.p2m.append(cheb.p2m(self.nc, c, h, self.points[ip], self.w[ip]))
            self.l2p.append(cheb.l2p(self.nc, c, h, self.points[ip]))
        self._m2m = {}
        self._m2l = {}

    def m2m(self, lvl, i):
        key = tuple(int(v) & 1 for v in self.tree.levels[lvl].coords[i])
        if key not in self._m2m:
            self._m2m[key] = cheb.m2m(self.nc, _octant(self.tree.levels[lvl].coords[i]))
        return self._m2m[key]

    def m2l(self, lvl, t, s):
        """M2L of the pair; it depends only on the level and the box offset, so
        the first pair of each (level, offset) is evaluated and reused."""
        T = self.tree
        key = (lvl,) + tuple(int(v) for v in (T.levels[lvl].coords[s] - T.levels[lvl].coords[t]))
        if key not in self._m2l:
            ct, h = T.box(lvl, t)
            cs, _ = T.box(lvl, s)
            self._m2l[key] = cheb.m2l(self.nc, ct, cs, h)
        return self._m2l[key]

    def matvec(self, x):
        T = self.tree
        L = T.depth
        x = np.asarray(x, dtype=np.float64)
        vec = x.ndim == 1
        X = x[:, None] if vec else x
        K = self.nc ** 3
        # upward pass
        mult = {L: [self.p2m[i] @ X[T.leaf_points(i)] for i in range(T.levels[L].n)]}
        for lvl in range(L - 1, 1, -1):
            lev = T.levels[lvl]
            mult[lvl] = [np.zeros((K, X.shape[1])) for _ in range(lev.n)]
            for c in range(T.levels[lvl + 1].n):
                p = T.levels[lvl + 1].parent[c]
                mult[lvl][p] += self.m2m(lvl + 1, c) @ mult[lvl + 1][c]
        # transfer at every level, then downward
        loc = {}
        for lvl in range(2, L + 1):
            lev = T.levels[lvl]
            loc[lvl] = []
            for i in range(lev.n):
                acc = np.zeros((K, X.shape[1]))
                for s in lev.il[i]:
                    acc += self.m2l(lvl, i, s) @ mult[lvl][s]
                if lvl > 2:
                    p = lev.parent[i]
                    acc += self.m2m(lvl, i).T @ loc[lvl - 1][p]
                loc[lvl].append(acc)
        # leaves: far field plus near field
        Y = np.zeros_like(X)
        leaf = T.levels[L]
        for i in range(leaf.n):
            ip = T.leaf_points(i)
            y = self.l2p[i] @ loc[L][i]
            for q in [i] + list(leaf.nbr[i]):
                iq = T.leaf_points(q)
                blk = cheb.p2p(self.points[ip], self.points[iq], self.w[iq], diag_t=self.diag[ip], same=(q == i))
                y = y + blk @ X[iq]
            Y[ip] = y
        return Y[:, 0] if vec else Y
