"""Oracle: the block-diagonal preconditioner BD of Sec. 4.3.

Test infrastructure only (see the package header).

BD (bottom level l_BD) groups the points by the boxes of level l_BD of the
uniform octree (the same root cube and box keys as the IFMM's tree) and
applies the inverse of the diagonal blocks of A: for every box b,
    z_b = A_bb^-1 r_b,   A_bb = A restricted to the points of box b,
where A_ij = K(p_i, p_j) w_j (i != j) and A_ii = diag_i.  The paper's leaf
BD takes l_BD = the leaf level; a coarser l_BD gives wider blocks.  Each
block is solved with LAPACK's LU (scipy), as written.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .tree import Tree


class BD:
    def __init__(self, points, diag, weights=None, level=0, leaf_max=64):
        points = np.asarray(points, dtype=np.float64)
        self.N = points.shape[0]
        w = np.ones(self.N) if weights is None else np.asarray(weights, dtype=np.float64)
        dg = np.full(self.N, float(diag)) if np.isscalar(diag) else np.asarray(diag, dtype=np.float64)
        self.tree = Tree(points, leaf_max=leaf_max, sigma=3, depth=level)
        leaf = self.tree.levels[self.tree.depth]
        self.boxes = []
        for b in range(leaf.n):
            idx = self.tree.perm[leaf.pt_begin[b]:leaf.pt_end[b]]
            P = points[idx]
            r = np.linalg.norm(P[:, None, :] - P[None, :, :], axis=2)
            with np.errstate(divide="ignore"):
                A = w[idx][None, :] / (4.0 * np.pi * r)
            A[np.arange(len(idx)), np.arange(len(idx))] = dg[idx]
            self.boxes.append((idx, sla.lu_factor(A)))

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        z = np.empty_like(r)
        for idx, lu in self.boxes:
            z[idx] = sla.lu_solve(lu, r[idx])
        return z
