"""Oracle: octree, neighbour / interaction lists and greedy colouring.

Test infrastructure only (see the package header).

Paper passages followed:
* Sec. 2.1 (hierarchical domain decomposition): a uniform octree, nodes are
  the non-empty boxes of each level; neighbours are the adjacent boxes
  excluding the node itself; the interaction list holds the non-adjacent
  children of the neighbours of the parent.
* Sec. 3, normalised distance equation: dist(u, v) = max-norm distance of
  the box centres over the box side, 1 <=> neighbour, 2 or 3 <=> interaction
  list.
* Alg. 3 (colouring): greedy lexicographic scan with stride sigma, k outer,
  i inner.

Readings (the paper leaves these open):
* Root cube: the tight bounding cube of the points (centre = midpoint of the
  bounding box, half-side = half the largest extent).
* Box keys at depth l: clamp(floor((x - lo) * s), 0, 2^l - 1) with
  s = 2^l / (2 H) evaluated as single IEEE operations; coarser keys are the
  leaf keys shifted right.
* Depth: the smallest l >= 2 whose fullest leaf holds at most ``leaf_max``
  points.
* Node order at every level: lexicographic in (k, j, i) = (z, y, x) box
  coordinates; points are stably sorted by their leaf box in that order.
"""
from __future__ import annotations

import numpy as np


class Level:
    """The non-empty boxes of one octree level.

    coords[i]   -- integer (i, j, k) = (x, y, z) box coordinates of node i
    parent[i]   -- index of the parent node in the coarser level (-1 at level 2)
    children[i] -- indices of the child nodes in the finer level (sorted)
    nbr[i]      -- neighbour list N_i (dist == 1), sorted by node index
    il[i]       -- interaction list I_i (dist 2 or 3, parents adjacent), sorted
    colour[i]   -- colour from Alg. 3; groups[c] lists the nodes of colour c
    """

    def __init__(self, level: int, coords: np.ndarray):
        self.level = level
        self.coords = coords
        self.n = coords.shape[0]
        self.index = {tuple(int(v) for v in c): i for i, c in enumerate(coords)}
        self.parent = np.full(self.n, -1, dtype=np.int64)
        self.children = [[] for _ in range(self.n)]
        self.nbr = [[] for _ in range(self.n)]
        self.il = [[] for _ in range(self.n)]
        self.colour = None
        self.groups = None
        # leaf data
        self.pt_begin = None
        self.pt_end = None


def dist(a, b) -> int:
    """Normalised max-norm distance between two boxes of one level (Sec. 3)."""
    return int(max(abs(int(a[0]) - int(b[0])), abs(int(a[1]) - int(b[1])), abs(int(a[2]) - int(b[2]))))


def root_cube(points: np.ndarray):
    """Tight bounding cube: returns (lo (3,), H) with the cube [lo, lo + 2H]^3."""
    pmin = points.min(axis=0)
    pmax = points.max(axis=0)
    centre = (pmin + pmax) / 2.0
    H = float(np.max(pmax - pmin)) / 2.0
    if not H > 0.0:
        raise ValueError("all points coincide: the root cube is empty")
    lo = centre - H
    return lo, H


def box_keys(points: np.ndarray, lo: np.ndarray, H: float, level: int) -> np.ndarray:
    """Integer box coordinates of every point at `level` (one IEEE op per step)."""
    m = 1 << level
    s = float(m) / (2.0 * H)
    keys = np.empty(points.shape, dtype=np.int64)
    for d in range(3):
        t = (points[:, d] - lo[d]) * s
        keys[:, d] = np.clip(np.floor(t), 0, m - 1).astype(np.int64)
    return keys


def lex_code(keys: np.ndarray, level: int) -> np.ndarray:
    """Lexicographic (k, j, i) code of box coordinates (k = z slowest)."""
    m = 1 << level
    return (keys[:, 2] * m + keys[:, 1]) * m + keys[:, 0]


def choose_depth(points: np.ndarray, lo, H, leaf_max: int) -> int:
    level = 2
    while True:
        codes = lex_code(box_keys(points, lo, H, level), level)
        _, counts = np.unique(codes, return_counts=True)
        if counts.max() <= leaf_max:
            return level
        level += 1
        if level > 20:
            raise ValueError("could not reach the leaf size: too many coincident points")


def colour_grid(occupied: np.ndarray, sigma: int) -> np.ndarray:
    """Greedy sigma-stride colouring of one level (Sec. 3.4, Alg. 3).

    occupied[k, j, i] marks the non-empty boxes of an m x m x m level; the
    result holds colour[k, j, i] (-1 for empty boxes).

    The rule, as Sec. 3.4 states it: a colour starts at the first box, in
    (k, j, i) scan order, that is non-empty and not yet coloured (the seed).
    The rest of the grid is then walked in scan order from the seed.  A
    non-empty uncoloured box on the walk takes the colour, and the walk then
    jumps sigma boxes ahead along i instead of one.  Likewise a row (fixed k, j)
    in which the colour was placed is followed by the row sigma further on,
    and a plane (fixed k) in which it was placed by the plane sigma further on;
    otherwise the walk moves to the next row / plane.  The seed counts as a
    placement in its row and plane.  Colours are numbered in the order their
    seeds are found.
    """
    m = occupied.shape[0]
    colour = np.full(occupied.shape, -1, dtype=np.int64)

    def free(k, j, i):
        return bool(occupied[k, j, i]) and colour[k, j, i] < 0

    def walk_row(k, j, i, g):
        """Places colour g along row (k, j) from box i on; True if it placed any."""
        placed = False
        while i < m:
            if free(k, j, i):
                colour[k, j, i] = g
                placed = True
                i += sigma
            else:
                i += 1
        return placed

    g = 0
    for seed in range(m * m * m):  # scan order: i fastest, then j, then k
        k0, j0, i0 = seed // (m * m), (seed // m) % m, seed % m
        if not free(k0, j0, i0):
            continue
        colour[k0, j0, i0] = g
        k = k0
        while k < m:
            in_seed_plane = k == k0
            plane_placed = in_seed_plane
            j = j0 if in_seed_plane else 0
            while j < m:
                if in_seed_plane and j == j0:
                    row_placed = walk_row(k, j, i0 + sigma, g) or True  # the seed's row
                else:
                    row_placed = walk_row(k, j, 0, g)
                plane_placed = plane_placed or row_placed
                j += sigma if row_placed else 1
            k += sigma if plane_placed else 1
        g += 1
    return colour


def colour_lookback(coords: np.ndarray, sigma: int) -> np.ndarray:
    """Greedy colouring that looks back at the boxes already coloured (the
    improvement Sec. 3.4 names in its closing remark and Sec. 6 leaves open).

    coords: (n, 3) integer box coordinates in (k, j, i) scan order.  Each
    colour walks all uncoloured boxes in scan order and takes every box whose
    distance (largest coordinate difference) to every box it already holds is
    at least sigma; the first uncoloured box always qualifies.  Same-colour
    boxes are then sigma-separated by construction.
    """
    n = coords.shape[0]
    colour = np.full(n, -1, dtype=np.int64)
    g = 0
    while np.any(colour < 0):
        members = np.empty((0, 3), dtype=coords.dtype)
        for i in range(n):
            if colour[i] >= 0:
                continue
            if members.shape[0] == 0 or np.min(np.max(np.abs(members - coords[i]), axis=1)) >= sigma:
                colour[i] = g
                members = np.vstack([members, coords[i]])
        g += 1
    return colour


def colour_level(lev: Level, sigma: int, tau: int = 2, colouring: str = "stride"):
    """Colours of one level: one node per colour below tau (the levels
    eliminated one node at a time), else Alg. 3 ("stride") or the look-back
    greedy ("lookback")."""
    m = 1 << lev.level
    c = lev.coords
    if lev.level < tau:
        lev.colour = np.arange(lev.n, dtype=np.int64)
    elif colouring == "lookback":
        lev.colour = colour_lookback(c, sigma)
    else:
        occ = np.zeros((m, m, m), dtype=bool)
        occ[c[:, 2], c[:, 1], c[:, 0]] = True
        grid = colour_grid(occ, sigma)
        lev.colour = grid[c[:, 2], c[:, 1], c[:, 0]].copy()
    ng = int(lev.colour.max()) + 1 if lev.n else 0
    # nodes are in (k, j, i) order, which is also the order Alg. 3 assigns them
    lev.groups = [[] for _ in range(ng)]
    for i in range(lev.n):
        lev.groups[int(lev.colour[i])].append(i)


class Tree:
    """Uniform octree over a point set.

    perm[t] = original index of the t-th point in tree order; levels[l] for
    l = 2 .. depth (entries 0 and 1 are None).
    """

    def __init__(self, points: np.ndarray, leaf_max: int = 64, sigma: int = 6, depth: int = 0, tau: int = 2,
                 colouring: str = "stride"):
        points = np.asarray(points, dtype=np.float64)
        if points.ndim != 2 or points.shape[1] != 3 or points.shape[0] < 1:
            raise ValueError("points must be an (N, 3) array with N >= 1")
        if not np.all(np.isfinite(points)):
            raise ValueError("non-finite coordinates")
        self.points = points
        self.lo, self.H = root_cube(points)
        self.depth = depth if depth >= 2 else choose_depth(points, self.lo, self.H, leaf_max)
        L = self.depth
        keys = box_keys(points, self.lo, self.H, L)
        codes = lex_code(keys, L)
        self.perm = np.argsort(codes, kind="stable")
        self.levels = [None] * (L + 1)
        sorted_codes = codes[self.perm]
        sorted_keys = keys[self.perm]
        # leaf level
        uniq, first = np.unique(sorted_codes, return_index=True)
        leaf = Level(L, sorted_keys[first].copy())
        leaf.pt_begin = first.astype(np.int64)
        leaf.pt_end = np.append(first[1:], len(sorted_codes)).astype(np.int64)
        self.levels[L] = leaf
        # coarser levels: shift keys
        for lvl in range(L - 1, 1, -1):
            ck = self.levels[lvl + 1].coords >> 1
            cc = lex_code(ck, lvl)
            u, f = np.unique(cc, return_index=True)
            self.levels[lvl] = Level(lvl, ck[f].copy())
        for lvl in range(3, L + 1):
            fine, coarse = self.levels[lvl], self.levels[lvl - 1]
            for i in range(fine.n):
                p = coarse.index[tuple(int(v) for v in (fine.coords[i] >> 1))]
                fine.parent[i] = p
                coarse.children[p].append(i)
        for lvl in range(2, L + 1):
            self._lists(lvl)
            colour_level(self.levels[lvl], sigma, tau, colouring)
        self.sigma = sigma

    def _lists(self, lvl: int):
        """N_i and I_i by brute force over all node pairs of the level."""
        lev = self.levels[lvl]
        c = lev.coords
        for i in range(lev.n):
            d = np.max(np.abs(c - c[i]), axis=1)
            lev.nbr[i] = [int(v) for v in np.nonzero(d == 1)[0]]
            cand = np.nonzero(d >= 2)[0]
            if lvl == 2:
                # every level-1 box touches every other one
                lev.il[i] = [int(v) for v in cand]
            else:
                pc = c >> 1
                dp = np.max(np.abs(pc[cand] - pc[i]), axis=1)
                lev.il[i] = [int(v) for v in cand[dp <= 1]]

    def leaf_points(self, i: int) -> np.ndarray:
        """Original indices of the points of leaf i."""
        leaf = self.levels[self.depth]
        return self.perm[leaf.pt_begin[i]:leaf.pt_end[i]]

    def box(self, lvl: int, i: int):
        """(centre (3,), half-side) of node i at level lvl."""
        side = 2.0 * self.H / float(1 << lvl)
        c = self.lo + (self.levels[lvl].coords[i].astype(np.float64) + 0.5) * side
        return c, side / 2.0
