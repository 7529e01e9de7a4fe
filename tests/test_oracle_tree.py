"""Pins of the oracle's octree, lists and colouring (Alg. 3)."""
import itertools
import os

import numpy as np
import pytest

import synth
from oracle.tree import Tree, colour_grid, dist

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def sphere_occupancy(level):
    """Boxes of [-0.5, 0.5]^3 that the sphere |x| = 0.5 passes through."""
    m = 1 << level
    side = 1.0 / m
    lo = -0.5 + np.arange(m) * side
    hi = lo + side
    mn = np.where(lo > 0, lo, np.where(hi < 0, -hi, 0.0))
    mx = np.maximum(np.abs(lo), np.abs(hi))
    dmin = np.sqrt(mn[:, None, None] ** 2 + mn[None, :, None] ** 2 + mn[None, None, :] ** 2)
    dmax = np.sqrt(mx[:, None, None] ** 2 + mx[None, :, None] ** 2 + mx[None, None, :] ** 2)
    return (dmin < 0.5) & (dmax > 0.5)


def load_table2():
    rows = []
    with open(os.path.join(GOLDEN, "table2_sphere_colouring.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            lv, nodes, groups, mn, avg, mx = line.split()
            rows.append((int(lv), int(nodes), int(groups), int(mn), float(avg), int(mx)))
    return rows


@pytest.mark.parametrize("row", load_table2())
def test_table2_sigma3(row):
    lv, nodes, groups, mn, avg, mx = row
    occ = sphere_occupancy(lv)
    assert occ.sum() == nodes
    col = colour_grid(occ, 3)
    sizes = np.bincount(col[occ])
    assert len(sizes) == groups
    assert sizes.min() == mn and sizes.max() == mx
    assert abs(sizes.mean() - avg) < 5e-7


def _check_separation(col, occ, sigma):
    idx = np.argwhere(occ)
    c = col[occ]
    for a in range(len(idx)):
        same = c == c[a]
        same[a] = False
        if same.any():
            d = np.max(np.abs(idx[same] - idx[a]), axis=1)
            assert d.min() >= sigma


@pytest.mark.parametrize("sigma", [3, 4, 6])
def test_separation_random(sigma):
    rng = np.random.default_rng(sigma)
    for level in (3, 4):
        m = 1 << level
        occ = rng.random((m, m, m)) < 0.3
        col = colour_grid(occ, sigma)
        assert np.all(col[occ] >= 0) and np.all(col[~occ] == -1)
        _check_separation(col, occ, sigma)


@pytest.mark.parametrize("sigma", [3, 6])
def test_full_grid_is_optimal(sigma):
    # Sec. 3.4: on a complete level the colouring has sigma^3 colours, each a
    # stride-sigma sub-grid.
    m = 16
    occ = np.ones((m, m, m), dtype=bool)
    col = colour_grid(occ, sigma)
    assert col.max() + 1 == sigma ** 3
    for k, j, i in itertools.product(range(m), repeat=3):
        assert col[k, j, i] == col[k % sigma, j % sigma, i % sigma]


def test_fig5a_plane():
    # Fig. 5(a): one full 8 x 8 plane at sigma = 3 takes sigma^2 = 9 colours.
    occ = np.zeros((8, 8, 8), dtype=bool)
    occ[0] = True
    col = colour_grid(occ, 3)
    assert col.max() + 1 == 9


def test_lists_and_dependency_invariants():
    pts = synth.sphere_points(3000, 11)
    for sigma in (3, 6):
        T = Tree(pts, leaf_max=16, sigma=sigma)
        for lvl in range(2, T.depth + 1):
            lev = T.levels[lvl]
            c = lev.coords
            for i in range(lev.n):
                for v in lev.nbr[i]:
                    assert dist(c[i], c[v]) == 1 and i in lev.nbr[v]
                for v in lev.il[i]:
                    # normalised distance equation: 2 or 3 <=> interaction list
                    assert dist(c[i], c[v]) in (2, 3) and i in lev.il[v]
            # Sec. 3.1: sigma >= 3 => disjoint neighbour sets within a colour;
            # sigma >= 6 => no neighbour of i in the interaction list of a
            # neighbour of i' (the underlined updates never collide).
            for grp in lev.groups:
                seen = set()
                for i in grp:
                    nb = set(lev.nbr[i]) | {i}
                    assert not (nb & seen)
                    seen |= nb
                if sigma >= 6:
                    for a, b in itertools.combinations(grp, 2):
                        for q in lev.nbr[a]:
                            for q2 in lev.nbr[b]:
                                assert q2 not in lev.il[q]


def test_tree_partitions_points():
    pts = synth.ellipsoid_points(5000, 3, jitter=0.05)
    T = Tree(pts, leaf_max=20, sigma=3)
    leaf = T.levels[T.depth]
    counts = leaf.pt_end - leaf.pt_begin
    assert counts.sum() == len(pts) and counts.max() <= 20
    assert sorted(T.perm.tolist()) == list(range(len(pts)))
    # every point lies in (the closure of) its box
    for i in range(leaf.n):
        c, h = T.box(T.depth, i)
        p = pts[T.leaf_points(i)]
        assert np.all(np.abs(p - c) <= h * (1 + 1e-12))
    # depth is minimal
    if T.depth > 2:
        T2 = Tree.__new__(Tree)
        from oracle.tree import box_keys, lex_code
        codes = lex_code(box_keys(pts, T.lo, T.H, T.depth - 1), T.depth - 1)
        assert np.unique(codes, return_counts=True)[1].max() > 20


@pytest.mark.parametrize("sigma", [3, 4, 5, 6])
def test_lookback_colouring_is_separated_and_not_worse(sigma):
    # the look-back greedy: every colour sigma-separated (brute force), every
    # box coloured, and on sphere-like occupancies no more colours than Alg. 3
    from oracle.tree import colour_lookback
    rng = np.random.default_rng(10 + sigma)
    for level in (3, 4):
        m = 1 << level
        occ = rng.random((m, m, m)) < 0.3
        kk, jj, ii = np.nonzero(occ)
        coords = np.stack([ii, jj, kk], axis=1)  # np.nonzero walks (k, j, i) in scan order
        col = colour_lookback(coords, sigma)
        assert np.all(col >= 0)
        grid = np.full(occ.shape, -1)
        grid[kk, jj, ii] = col
        _check_separation(grid, occ, sigma)
    for level in (3, 4, 5):
        occ = sphere_occupancy(level)
        kk, jj, ii = np.nonzero(occ)
        coords = np.stack([ii, jj, kk], axis=1)
        n_lb = colour_lookback(coords, sigma).max() + 1
        n_a3 = colour_grid(occ, sigma).max() + 1
        assert n_lb <= n_a3, (level, n_lb, n_a3)


def test_lookback_full_grid_and_a_case_alg3_misses():
    from oracle.tree import colour_lookback
    m = 9
    coords = np.array([(i, j, k) for k in range(m) for j in range(m) for i in range(m)])
    col = colour_lookback(coords, 3)
    assert col.max() + 1 == 27
    # two boxes of one plane, (0, 0) and (5, 1) in (i, j), sigma = 3: Alg. 3
    # jumps three rows after the row of the seed and misses the second box;
    # looking back, it is 5 boxes from the seed and joins the first colour
    occ = np.zeros((8, 8, 8), dtype=bool)
    occ[0, 0, 0] = True
    occ[0, 1, 5] = True
    assert colour_grid(occ, 3).max() + 1 == 2
    assert colour_lookback(np.array([(0, 0, 0), (5, 1, 0)]), 3).max() + 1 == 1
