"""Oracle: the IFMM extended sparse system, its colour-ordered factorisation and solve.

Test infrastructure only (see the package header).  Plain FP64 numpy/scipy;
scipy's getrf/getrs (LU with partial pivoting) and numpy's SVD serve as steps.

What it follows
---------------
* Eq. (ext), Sec. 2.2: every node i carries particle unknowns x_i (n_i of them;
  for an internal node these are its children's multipole unknowns), multipole
  unknowns y_i and local unknowns z_i (r_i each).  Its rows are
      R_x:  sum_j P2P_ij x_j + L2P_i z_i = b_i
      R_y:  P2M_i x_i - y_i = 0
      R_z:  -z_i + sum_{l in I_i} M2L_il y_l + L2L_i z_parent = 0
  and a parent's R_x rows / C_x columns are its children's R_z rows / C_y
  columns, so its P2P, P2M and L2P are built from the children's M2L, M2M and
  L2L (Alg. 1, aggregation step).
* Alg. 1: levels from the leaves up; per node, block Gaussian elimination of
  the pivot (rows R_x, R_y; columns C_x, C_z), fill-in among the neighbours
  (Cases 1-4), low-rank compression of the fill-in between neighbours that
  lie in each other's interaction list, updates of the bases, of the M2L
  operators of their interaction lists and of M2M / L2L; then aggregation.
* Sec. 3.2 / 3.3: the node loop of a level is replaced by a serial loop over
  the colours of Alg. 3 and a loop over the nodes of one colour.
* Sec. 2.3 (last paragraph): after level 2 the remaining M2L system is solved
  densely with LU.
* Alg. 2: forward substitution in elimination order, the dense top solve,
  backward substitution in exactly the reverse order (colours descending).

Readings (the paper only sketches the IFMM and defers to its references)
------------------------------------------------------------------------
R1  Pivot.  D_i = [[P2P_ii, L2P_i], [P2M_i, 0]] over rows (R_x_i, R_y_i) and
    columns (C_x_i, C_z_i); the survivors of node i are its row R_z_i and
    column C_y_i.  After elimination the coupling between neighbours p and q
    is P2P_pq, M2P_pq, P2L_pq or M2L_pq depending on which of them is
    eliminated; the elimination of i adds M2P/M2L_pi = B_pi F,
    P2L/M2L_iq = (D^-1 U)_bottom and M2L_ii = -H, with [F; H] = D^-1 [0; I].
R2  Far fill-in (neighbours p, q of i with dist(p, q) = 2, hence q in I_p) is
    not stored.  For every non-eliminated neighbour p that receives any, all of
    its far fill-in of this elimination is compressed at once (Alg. 1 does it
    pair by pair; both are exact as eps -> 0):
      source side  W = [diag(sig_s) P2M_p ; F_qp ...]      (rows act on x_p)
      target side  W = [L2P_p diag(sig_t) , F_pq ...]      (columns act on x_p)
    An SVD of each keeps the singular values > eps * sigma_1 (strict); the new
    rank is the larger of the two counts (the pivot must stay square), capped
    by n_p and by an optional rank cap.  New bases are the leading singular
    vectors, new weights their singular values; T_p = P2M_p V', S_p = U'^T L2P_p.
R3  Weights.  sig_s / sig_t are node-local singular-value weights.  They start
    from the initial rank reduction, which compresses the Chebyshev P2M / L2P
    of a node (leaf, or freshly aggregated parent) against the far field it
    actually feeds:  G_i = sum_{l in I_i} M2L_li^T M2L_li + M2M_i^T G_par M2M_i
    (source) and H_i = sum_l M2L_il M2L_il^T + L2L_i H_par L2L_i^T (target),
    built top-down from the Chebyshev operators; the SVD is taken of
    G_i^(1/2) P2M_i and L2P_i H_i^(1/2) with the same truncation rule.  This
    makes the pivot square (r_i <= n_i), which the paper does not discuss.
R4  Colour semantics.  Within a colour every node does its elimination and
    compression first ("phase A"); the basis changes are then pushed into the
    M2L blocks of the interaction lists and into M2M / L2L, and the projected
    fill-ins added ("phase B").  Phase A reads nothing that phase B writes, so
    this equals applying the underlined updates of Alg. 1 immediately, and the
    result does not depend on the order inside a colour (the paper serialises
    those updates with an unordered critical section instead).
R5  Top level.  Level 2 is eliminated like any other level; the survivors
    (R_z, C_y of the level-2 nodes) form the dense system of all level-2 M2L
    blocks, which is LU-factorised.  Level-1 boxes have no interaction list,
    so no L2L term from level 1 appears.
R6  Ties: LU pivoting takes the largest |entry|, first on ties (LAPACK);
    the truncation count uses a strict '>'.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import cheb
from .tree import Tree, dist


def _trunc(s: np.ndarray, eps: float) -> int:
    if s.size == 0 or not s[0] > 0.0:
        return 0
    return int(np.count_nonzero(s > eps * s[0]))


def _pad(s: np.ndarray, r: int) -> np.ndarray:
    out = np.zeros(r)
    k = min(r, s.size)
    out[:k] = s[:k]
    return out


def _sqrt_psd(G: np.ndarray) -> np.ndarray:
    """Symmetric square root of a positive semi-definite matrix (eigenvalues
    clipped at 0)."""
    G = 0.5 * (G + G.T)
    lam, Q = np.linalg.eigh(G)
    lam = np.clip(lam, 0.0, None)
    return (Q * np.sqrt(lam)[None, :]) @ Q.T


def _right_svd(W: np.ndarray):
    """Singular values and a full set of right singular vectors (rows of Vt,
    n x n) of W (m x n)."""
    full = W.shape[0] < W.shape[1]
    _, s, Vt = np.linalg.svd(W, full_matrices=full)
    return s, Vt


def _left_svd(W: np.ndarray):
    """Singular values and a full set of left singular vectors (m x m) of W (m x n)."""
    full = W.shape[1] < W.shape[0]
    U, s, _ = np.linalg.svd(W, full_matrices=full)
    return U, s


def _octant(coord) -> np.ndarray:
    return np.array([2 * (int(c) & 1) - 1 for c in coord], dtype=np.float64)


class IFMM:
    """Factorisation of the extended system of an N x N Laplace matrix.

    points   (N, 3)  source = target points
    weights  (N,)    column scaling w_j (quadrature weights), default 1
    diag     (N,) or scalar: A_ii
    eps      relative truncation threshold (R2, R3)
    sigma    colouring separation (Alg. 3)
    """

    def __init__(self, points, eps=1e-6, sigma=6, leaf_max=64, cheb_order=4,
                 weights=None, diag=None, rank_cap=0, depth=0, tau=2, colouring="stride"):
        points = np.asarray(points, dtype=np.float64)
        N = points.shape[0]
        self.N = N
        self.points = points
        self.w = np.ones(N) if weights is None else np.asarray(weights, dtype=np.float64)
        if diag is None:
            raise ValueError("a diagonal (scalar or per point) is required")
        self.diag = np.full(N, float(diag)) if np.isscalar(diag) else np.asarray(diag, dtype=np.float64)
        if not (0.0 < eps < 1.0):
            raise ValueError("eps must lie in (0, 1)")
        if sigma < 3:
            raise ValueError("sigma must be >= 3")
        self.eps = float(eps)
        self.nc = int(cheb_order)
        self.K = self.nc ** 3
        self.rank_cap = int(rank_cap)
        self.tree = Tree(points, leaf_max=leaf_max, sigma=sigma, depth=depth, tau=tau, colouring=colouring)
        self.depth = self.tree.depth
        self.factored = False
        self._m2m_unit = {}

    # ------------------------------------------------------------------ operators
    def m2m_unit(self, coord) -> np.ndarray:
        key = tuple(int(c) & 1 for c in coord)
        if key not in self._m2m_unit:
            self._m2m_unit[key] = cheb.m2m(self.nc, _octant(coord))
        return self._m2m_unit[key]

    def m2l_cheb(self, lvl, t, s) -> np.ndarray:
        ct, h = self.tree.box(lvl, t)
        cs, _ = self.tree.box(lvl, s)
        return cheb.m2l(self.nc, ct, cs, h)

    def leaf_p2m(self, i):
        c, h = self.tree.box(self.depth, i)
        idx = self.tree.leaf_points(i)
        return cheb.p2m(self.nc, c, h, self.points[idx], self.w[idx])

    def leaf_l2p(self, i):
        c, h = self.tree.box(self.depth, i)
        idx = self.tree.leaf_points(i)
        return cheb.l2p(self.nc, c, h, self.points[idx])

    def leaf_p2p(self, p, q):
        ip = self.tree.leaf_points(p)
        iq = self.tree.leaf_points(q)
        if p == q:
            return cheb.p2p(self.points[ip], self.points[iq], self.w[iq], diag_t=self.diag[ip], same=True)
        return cheb.p2p(self.points[ip], self.points[iq], self.w[iq])

    # ------------------------------------------------------------------ weights (R3)
    def _weights(self):
        """Source / target far-field weights G, H per node, top-down (R3)."""
        T = self.tree
        self.Gw = [None] * (self.depth + 1)
        self.Hw = [None] * (self.depth + 1)
        for lvl in range(2, self.depth + 1):
            lev = T.levels[lvl]
            Gs, Hs = [], []
            for i in range(lev.n):
                G = np.zeros((self.K, self.K))
                H = np.zeros((self.K, self.K))
                for l in lev.il[i]:
                    Mli = self.m2l_cheb(lvl, l, i)   # source i -> target l
                    Mil = self.m2l_cheb(lvl, i, l)   # source l -> target i
                    G += Mli.T @ Mli
                    H += Mil @ Mil.T
                if lvl > 2:
                    par = int(lev.parent[i])
                    M = self.m2m_unit(lev.coords[i])
                    G += M.T @ self.Gw[lvl - 1][par] @ M
                    H += M.T @ self.Hw[lvl - 1][par] @ M   # L2L = M2M^T
                Gs.append(G)
                Hs.append(H)
            self.Gw[lvl] = Gs
            self.Hw[lvl] = Hs

    # ------------------------------------------------------------------ level set-up
    def _reduce_level(self, lvl, P2Mc, L2Pc):
        """Initial rank reduction of every node of a level (R3), then the
        reduced M2L, M2M and L2L operators of the level."""
        lev = self.tree.levels[lvl]
        S_ = self.state[lvl]
        T_list, S_list = [], []
        for i in range(lev.n):
            n_i = P2Mc[i].shape[1]
            W0s = _sqrt_psd(self.Gw[lvl][i]) @ P2Mc[i]
            W0t = L2Pc[i] @ _sqrt_psd(self.Hw[lvl][i])
            ss, Vt = _right_svd(W0s)
            Ut, st = _left_svd(W0t)
            r = max(_trunc(ss, self.eps), _trunc(st, self.eps))
            r = min(r, n_i)
            if self.rank_cap > 0:
                r = min(r, self.rank_cap)
            V = Vt[:r].T
            U = Ut[:, :r]
            S_["P2M"][i] = V.T.copy()
            S_["L2P"][i] = U.copy()
            S_["sig_s"][i] = _pad(ss, r)
            S_["sig_t"][i] = _pad(st, r)
            S_["r"][i] = r
            T_list.append(P2Mc[i] @ V)        # K x r : y_cheb = T y
            S_list.append(U.T @ L2Pc[i])      # r x K : z = S z_cheb
        for i in range(lev.n):
            for l in lev.il[i]:
                S_["m2l"][(i, l)] = S_list[i] @ self.m2l_cheb(lvl, i, l) @ T_list[l]
            if lvl > 2:
                M = self.m2m_unit(lev.coords[i])
                S_["M2M"][i] = M @ T_list[i]          # parent cheb <- y_i
                S_["L2L"][i] = S_list[i] @ M.T        # z_i <- parent cheb

    def _new_state(self, lvl):
        n = self.tree.levels[lvl].n
        return {"n": np.zeros(n, dtype=np.int64), "r": np.zeros(n, dtype=np.int64),
                "elim": np.zeros(n, dtype=bool), "near": {}, "m2l": {},
                "P2M": [None] * n, "L2P": [None] * n, "sig_s": [None] * n, "sig_t": [None] * n,
                "M2M": [None] * n, "L2L": [None] * n}

    def _init_leaves(self):
        L = self.depth
        lev = self.tree.levels[L]
        S_ = self._new_state(L)
        self.state[L] = S_
        for i in range(lev.n):
            S_["n"][i] = lev.pt_end[i] - lev.pt_begin[i]
            S_["near"][(i, i)] = self.leaf_p2p(i, i)
            for q in lev.nbr[i]:
                S_["near"][(i, q)] = self.leaf_p2p(i, q)
        P2Mc = [self.leaf_p2m(i) for i in range(lev.n)]
        L2Pc = [self.leaf_l2p(i) for i in range(lev.n)]
        self._reduce_level(L, P2Mc, L2Pc)

    def _aggregate(self, lvl):
        """Alg. 1, aggregation: level lvl (all eliminated) -> level lvl - 1."""
        fine = self.tree.levels[lvl]
        coarse = self.tree.levels[lvl - 1]
        Sf = self.state[lvl]
        Sc = self._new_state(lvl - 1)
        self.state[lvl - 1] = Sc

        def blk(c, cc):
            if dist(fine.coords[c], fine.coords[cc]) <= 1:
                return Sf["near"][(c, cc)]
            return Sf["m2l"][(c, cc)]

        P2Mc, L2Pc = [], []
        for P in range(coarse.n):
            ch = coarse.children[P]
            Sc["n"][P] = int(sum(Sf["r"][c] for c in ch))
            P2Mc.append(np.hstack([Sf["M2M"][c] for c in ch]))
            L2Pc.append(np.vstack([Sf["L2L"][c] for c in ch]))
            for Q in [P] + coarse.nbr[P]:
                chQ = coarse.children[Q]
                rows = [np.hstack([blk(c, cc) for cc in chQ]) for c in ch]
                Sc["near"][(P, Q)] = np.vstack(rows)
        self._reduce_level(lvl - 1, P2Mc, L2Pc)
        # the fine level's working blocks are no longer needed
        Sf["near"] = None
        Sf["m2l"] = None

    # ------------------------------------------------------------------ phase A
    def _eliminate(self, lvl, i, pend_basis, pend_add):
        lev = self.tree.levels[lvl]
        S_ = self.state[lvl]
        near = S_["near"]
        n_i, r_i = int(S_["n"][i]), int(S_["r"][i])
        d = n_i + r_i
        D = np.zeros((d, d))
        D[:n_i, :n_i] = near[(i, i)]
        D[:n_i, n_i:] = S_["L2P"][i]
        D[n_i:, :n_i] = S_["P2M"][i]
        nb = lev.nbr[i]
        was_elim = {p: bool(S_["elim"][p]) for p in nb}
        Lb = [near[(p, i)].copy() for p in nb]     # B_pi: rows of p, columns x_i
        Ub = [near[(i, q)].copy() for q in nb]     # B_iq: rows x_i, columns of q
        widths = [B.shape[1] for B in Ub]
        offs = np.concatenate([[0], np.cumsum(widths)]).astype(int)
        Wd = int(offs[-1])
        rec = {"n": n_i, "r": r_i, "nbr": list(nb),
               "kind": ["z" if was_elim[p] else "x" for p in nb], "L": Lb, "U": Ub}
        if d > 0:
            lu = sla.lu_factor(D)
            rhs = np.zeros((d, Wd + r_i))
            if Wd:
                rhs[:n_i, :Wd] = np.hstack(Ub)
            rhs[n_i:, Wd:] = np.eye(r_i)
            X = sla.lu_solve(lu, rhs)
        else:
            lu = None
            X = np.zeros((0, Wd))
        rec["lu"] = lu
        Xtop, Xbot = X[:n_i], X[n_i:]
        F = Xtop[:, Wd:]
        Hm = Xbot[:, Wd:]
        far = {}
        for a, p in enumerate(nb):
            for b, q in enumerate(nb):
                C = Lb[a] @ Xtop[:, offs[b]:offs[b + 1]]
                if dist(lev.coords[p], lev.coords[q]) <= 1:
                    near[(p, q)] = near[(p, q)] - C
                else:
                    far[(p, q)] = -C
        for a, p in enumerate(nb):
            near[(p, i)] = Lb[a] @ F
        for b, q in enumerate(nb):
            near[(i, q)] = Xbot[:, offs[b]:offs[b + 1]].copy()
        near[(i, i)] = -Hm
        S_["elim"][i] = True
        self.rec[lvl][i] = rec
        # compression of far fill-in (R2)
        newb = {}
        for p in nb:
            if was_elim[p]:
                continue
            Qp = [q for q in nb if (p, q) in far]
            if not Qp:
                continue
            n_p = int(S_["n"][p])
            Wsrc = np.vstack([S_["sig_s"][p][:, None] * S_["P2M"][p]] + [far[(q, p)] for q in Qp])
            Wtgt = np.hstack([S_["L2P"][p] * S_["sig_t"][p][None, :]] + [far[(p, q)] for q in Qp])
            ss, Vt = _right_svd(Wsrc)
            Ut, st = _left_svd(Wtgt)
            rn = max(_trunc(ss, self.eps), _trunc(st, self.eps))
            rn = min(rn, n_p)
            if self.rank_cap > 0:
                rn = min(rn, self.rank_cap)
            V = Vt[:rn].T
            U = Ut[:, :rn]
            newb[p] = {"V": V, "U": U, "sig_s": _pad(ss, rn), "sig_t": _pad(st, rn),
                       "T": S_["P2M"][p] @ V, "S": U.T @ S_["L2P"][p], "r": rn}
        for (p, q), Fpq in far.items():
            Dl = Fpq
            if not was_elim[p]:
                Dl = newb[p]["U"].T @ Dl
            if not was_elim[q]:
                Dl = Dl @ newb[q]["V"]
            pend_add[(p, q)] = Dl
        pend_basis.update(newb)

    # ------------------------------------------------------------------ phase B
    def _phase_b(self, lvl, pend_basis, pend_add):
        lev = self.tree.levels[lvl]
        S_ = self.state[lvl]
        m2l = S_["m2l"]
        keys = set()
        for p in pend_basis:
            for l in lev.il[p]:
                keys.add((l, p))
                keys.add((p, l))
        for (t, s) in sorted(keys):
            M = m2l[(t, s)]
            if t in pend_basis:
                M = pend_basis[t]["S"] @ M
            if s in pend_basis:
                M = M @ pend_basis[s]["T"]
            m2l[(t, s)] = M
        for key, Dl in pend_add.items():
            m2l[key] = m2l[key] + Dl
        for p, nbk in pend_basis.items():
            if lvl > 2:
                S_["M2M"][p] = S_["M2M"][p] @ nbk["T"]
                S_["L2L"][p] = nbk["S"] @ S_["L2L"][p]
            S_["P2M"][p] = nbk["V"].T.copy()
            S_["L2P"][p] = nbk["U"].copy()
            S_["sig_s"][p] = nbk["sig_s"]
            S_["sig_t"][p] = nbk["sig_t"]
            S_["r"][p] = nbk["r"]

    # ------------------------------------------------------------------ factor
    def factor(self, order=None):
        """Alg. 1 with the colour loops of Sec. 3.  `order`, if given, maps
        (level, colour) -> a permutation of the colour's nodes (to check that
        the order inside a colour does not matter)."""
        T = self.tree
        self._weights()
        self.state = [None] * (self.depth + 1)
        self.rec = [None] * (self.depth + 1)
        self._init_leaves()
        for lvl in range(self.depth, 1, -1):
            lev = T.levels[lvl]
            self.rec[lvl] = [None] * lev.n
            for c, grp in enumerate(lev.groups):
                nodes = list(grp)
                if order is not None:
                    nodes = list(order(lvl, c, nodes))
                pend_basis, pend_add = {}, {}
                for i in nodes:
                    self._eliminate(lvl, i, pend_basis, pend_add)
                self._phase_b(lvl, pend_basis, pend_add)
            if lvl > 2:
                self._aggregate(lvl)
        # top: dense system of all level-2 M2L blocks (R5)
        lev2 = T.levels[2]
        S2 = self.state[2]
        r2 = [int(S2["r"][P]) for P in range(lev2.n)]
        off = np.concatenate([[0], np.cumsum(r2)]).astype(int)
        Mtop = np.zeros((off[-1], off[-1]))
        for P in range(lev2.n):
            for Q in range(lev2.n):
                if dist(lev2.coords[P], lev2.coords[Q]) <= 1:
                    B = S2["near"][(P, Q)]
                else:
                    B = S2["m2l"][(P, Q)]
                Mtop[off[P]:off[P + 1], off[Q]:off[Q + 1]] = B
        self.top_off = off
        self.top = sla.lu_factor(Mtop) if off[-1] > 0 else None
        self.top_dense = Mtop
        self.factored = True
        return self

    # ------------------------------------------------------------------ solve
    def solve(self, b):
        """Alg. 2 with the colour order of the factorisation (reversed on the
        way back).  b: (N,) or (N, k) in the original point order."""
        if not self.factored:
            raise RuntimeError("factor() must run before solve()")
        T = self.tree
        b = np.asarray(b, dtype=np.float64)
        vec = b.ndim == 1
        B = b.reshape(self.N, -1)
        k = B.shape[1]
        L = self.depth
        Bp = B[T.perm]
        fx = [None] * (L + 1)
        fz = [None] * (L + 1)
        wv = [None] * (L + 1)
        leaf = T.levels[L]
        fx[L] = [Bp[leaf.pt_begin[i]:leaf.pt_end[i]].copy() for i in range(leaf.n)]
        for lvl in range(L, 1, -1):
            lev = T.levels[lvl]
            S_ = self.state[lvl]
            fz[lvl] = [np.zeros((int(S_["r"][i]), k)) for i in range(lev.n)]
            wv[lvl] = [None] * lev.n
            for grp in lev.groups:
                for i in grp:
                    rec = self.rec[lvl][i]
                    n_i, r_i = rec["n"], rec["r"]
                    piv = np.vstack([fx[lvl][i], np.zeros((r_i, k))])
                    w = sla.lu_solve(rec["lu"], piv) if rec["lu"] is not None else piv
                    wv[lvl][i] = w
                    for p, kind, Bl in zip(rec["nbr"], rec["kind"], rec["L"]):
                        if kind == "x":
                            fx[lvl][p] = fx[lvl][p] - Bl @ w[:n_i]
                        else:
                            fz[lvl][p] = fz[lvl][p] - Bl @ w[:n_i]
                    fz[lvl][i] = fz[lvl][i] + w[n_i:]
            if lvl > 2:
                coarse = T.levels[lvl - 1]
                fx[lvl - 1] = [np.vstack([fz[lvl][c] for c in coarse.children[P]] + [np.zeros((0, k))])
                               for P in range(coarse.n)]
        # top
        lev2 = T.levels[2]
        ftop = np.vstack([fz[2][P] for P in range(lev2.n)] + [np.zeros((0, k))])
        ytop = sla.lu_solve(self.top, ftop) if self.top is not None else ftop
        xx = [None] * (L + 1)
        xy = [None] * (L + 1)
        xy[2] = [ytop[self.top_off[P]:self.top_off[P + 1]] for P in range(lev2.n)]
        for lvl in range(2, L + 1):
            lev = T.levels[lvl]
            if lvl > 2:
                coarse = T.levels[lvl - 1]
                xy[lvl] = [None] * lev.n
                Sf = self.state[lvl]
                for P in range(coarse.n):
                    o = 0
                    for c in coarse.children[P]:
                        rc = int(Sf["r"][c])
                        xy[lvl][c] = xx[lvl - 1][P][o:o + rc]
                        o += rc
            xx[lvl] = [None] * lev.n
            for grp in reversed(lev.groups):
                for i in grp:
                    rec = self.rec[lvl][i]
                    n_i, r_i = rec["n"], rec["r"]
                    ub = np.zeros((n_i, k))
                    for q, kind, Bu in zip(rec["nbr"], rec["kind"], rec["U"]):
                        xq = xx[lvl][q] if kind == "x" else xy[lvl][q]
                        ub = ub + Bu @ xq
                    rhs = np.vstack([ub, -xy[lvl][i]])
                    corr = sla.lu_solve(rec["lu"], rhs) if rec["lu"] is not None else rhs
                    piv = wv[lvl][i] - corr
                    xx[lvl][i] = piv[:n_i]
        out = np.empty_like(Bp)
        out[T.perm] = np.vstack([xx[L][i] for i in range(leaf.n)])
        return out[:, 0] if vec else out

    # ------------------------------------------------------------------ statistics
    def ranks(self):
        """Final rank of every node, per level."""
        return {lvl: self.state[lvl]["r"].copy() for lvl in range(2, self.depth + 1)}


def dense_tilde(points, weights, diag, leaf_max=64, cheb_order=4, sigma=6, depth=0):
    """The matrix the extended system represents exactly (tiny N only):
    near leaf pairs (dist <= 1) take A; every other leaf pair takes
    L2P (L2L chain) M2L (M2M chain) P2M at the level where the two ancestors
    lie in each other's interaction list."""
    points = np.asarray(points, dtype=np.float64)
    N = points.shape[0]
    w = np.ones(N) if weights is None else np.asarray(weights, dtype=np.float64)
    dg = np.full(N, float(diag)) if np.isscalar(diag) else np.asarray(diag, dtype=np.float64)
    T = Tree(points, leaf_max=leaf_max, sigma=sigma, depth=depth)
    L = T.depth
    nc = cheb_order
    leaf = T.levels[L]
    At = np.zeros((N, N))
    m2m8 = {}

    def m2m_of(lvl, i):
        key = tuple(int(c) & 1 for c in T.levels[lvl].coords[i])
        if key not in m2m8:
            m2m8[key] = cheb.m2m(nc, _octant(T.levels[lvl].coords[i]))
        return m2m8[key]

    # up[lvl][q]: x_q -> Chebyshev multipole of q's ancestor at lvl (M2M chain . P2M)
    # down[lvl][p]: Chebyshev local of p's ancestor at lvl -> potentials at p's points
    up = {L: [], }
    down = {L: []}
    anc = {L: list(range(leaf.n))}
    for p in range(leaf.n):
        ip = T.leaf_points(p)
        c, h = T.box(L, p)
        up[L].append(cheb.p2m(nc, c, h, points[ip], w[ip]))
        down[L].append(cheb.l2p(nc, c, h, points[ip]))
    for lvl in range(L - 1, 1, -1):
        up[lvl], down[lvl], anc[lvl] = [], [], []
        for p in range(leaf.n):
            a = anc[lvl + 1][p]
            M = m2m_of(lvl + 1, a)
            up[lvl].append(M @ up[lvl + 1][p])
            down[lvl].append(down[lvl + 1][p] @ M.T)
            anc[lvl].append(int(T.levels[lvl + 1].parent[a]))
    m2l_cache = {}
    for p in range(leaf.n):
        ip = T.leaf_points(p)
        for q in range(leaf.n):
            iq = T.leaf_points(q)
            if dist(leaf.coords[p], leaf.coords[q]) <= 1:
                blk = cheb.p2p(points[ip], points[iq], w[iq], diag_t=dg[ip], same=(p == q))
            else:
                lvl = L
                while lvl > 2:
                    pp = anc[lvl - 1][p]
                    qq = anc[lvl - 1][q]
                    if dist(T.levels[lvl - 1].coords[pp], T.levels[lvl - 1].coords[qq]) <= 1:
                        break
                    lvl -= 1
                P, Q = anc[lvl][p], anc[lvl][q]
                key = (lvl, P, Q)
                if key not in m2l_cache:
                    cP, h = T.box(lvl, P)
                    cQ, _ = T.box(lvl, Q)
                    m2l_cache[key] = cheb.m2l(nc, cP, cQ, h)
                blk = down[lvl][p] @ m2l_cache[key] @ up[lvl][q]
            At[np.ix_(ip, iq)] = blk
    return At
