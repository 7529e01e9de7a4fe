// Host octree, lists and colouring (see tree.hpp).  Compiled with
// -ffp-contract=off so that the box keys are reproducible bit for bit.
#include "tree.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <numeric>
#include <unordered_map>

namespace ifmm {

int Level::dist(int32_t a, int32_t b) const {
  int d = 0;
  for (int e = 0; e < 3; ++e) d = std::max(d, std::abs(coord[3 * a + e] - coord[3 * b + e]));
  return d;
}

static inline int64_t lex(int32_t i, int32_t j, int32_t k, int64_t m) { return ((int64_t)k * m + j) * m + i; }

// Greedy sigma-stride colouring of one level (Sec. 3.4, Alg. 3).  The rule:
// a colour starts at the first non-empty uncoloured box in (k, j, i) scan
// order and walks the rest of the grid in scan order; a box it colours makes
// the walk continue sigma boxes further along i, a row in which it coloured a
// box is followed by the row sigma further on, a plane likewise by the plane
// sigma further on (otherwise the next row / plane); the seed counts as a
// placement in its row and plane.
//
// Only occupied boxes are stored: every row (k, j) keeps its uncoloured boxes
// as an ascending list of i.  Walking a row from i = start takes the first
// listed box at or after start, then the first at or after that box + sigma,
// and so on, which is what the box-by-box walk does.
int32_t colour_grid(const std::vector<uint8_t>& occ, int m, int sigma, std::vector<int32_t>& colour) {
  const int64_t M = m;
  colour.assign((size_t)(M * M * M), -1);
  std::vector<std::vector<int32_t>> row_free((size_t)(M * M));
  for (int64_t r = 0; r < M * M; ++r)
    for (int32_t i = 0; i < m; ++i)
      if (occ[(size_t)(r * M + i)]) row_free[(size_t)r].push_back(i);
  // colours row r = k m + j from i = start on; returns whether it placed any
  auto walk_row = [&](int64_t r, int32_t start, int32_t g) {
    std::vector<int32_t>& list = row_free[(size_t)r];
    size_t keep = 0;
    bool placed = false;
    for (size_t t = 0; t < list.size(); ++t) {
      const int32_t i = list[t];
      if (i >= start) {
        colour[(size_t)(r * M + i)] = g;
        placed = true;
        start = i + sigma;
      } else {
        list[keep++] = i;
      }
    }
    list.resize(keep);
    return placed;
  };
  int32_t g = 0;
  int64_t seed_row = 0;
  for (;;) {
    while (seed_row < M * M && row_free[(size_t)seed_row].empty()) ++seed_row;
    if (seed_row == M * M) break;
    const int32_t k0 = (int32_t)(seed_row / M), j0 = (int32_t)(seed_row % M);
    // the seed: first free box of the first row that has one
    std::vector<int32_t>& first = row_free[(size_t)seed_row];
    const int32_t i0 = first.front();
    colour[(size_t)(seed_row * M + i0)] = g;
    first.erase(first.begin());
    for (int32_t k = k0; k < m;) {
      const bool seed_plane = k == k0;
      bool plane_placed = seed_plane;
      for (int32_t j = seed_plane ? j0 : 0; j < m;) {
        const int64_t r = (int64_t)k * M + j;
        const bool seed_row_here = seed_plane && j == j0;
        const bool row_placed = walk_row(r, seed_row_here ? i0 + sigma : 0, g) || seed_row_here;
        plane_placed = plane_placed || row_placed;
        j += row_placed ? sigma : 1;
      }
      k += plane_placed ? sigma : 1;
    }
    ++g;
  }
  return g;
}

// Greedy colouring that looks back at the boxes already coloured: each colour
// walks the uncoloured nodes in scan order (node order) and takes every node
// at distance >= sigma from all nodes it already holds.  A placed node blocks
// the (2 sigma - 1)^3 boxes around it for the current colour (a stamp grid),
// so the test is one lookup per candidate.
int32_t colour_lookback(const Level& lv, int m, int sigma, std::vector<int32_t>& colour) {
  const int64_t M = m;
  colour.assign((size_t)lv.n, -1);
  std::vector<int32_t> stamp((size_t)(M * M * M), 0);
  int32_t g = 0, left = lv.n;
  while (left > 0) {
    for (int32_t i = 0; i < lv.n; ++i) {
      if (colour[i] >= 0) continue;
      const int x = lv.coord[3 * i], y = lv.coord[3 * i + 1], z = lv.coord[3 * i + 2];
      if (stamp[(size_t)lex(x, y, z, M)] == g + 1) continue;
      colour[i] = g;
      --left;
      for (int k = std::max(0, z - sigma + 1); k <= std::min(m - 1, z + sigma - 1); ++k)
        for (int j = std::max(0, y - sigma + 1); j <= std::min(m - 1, y + sigma - 1); ++j)
          for (int q = std::max(0, x - sigma + 1); q <= std::min(m - 1, x + sigma - 1); ++q)
            stamp[(size_t)lex(q, j, k, M)] = g + 1;
    }
    ++g;
  }
  return g;
}

// Cost model of the bottom level (Sec. 5.2: the leaf-level cost grows with
// the number of leaf nodes times the cube of their block sizes, so removing
// fine levels pays until the leaves get too large).  Candidate depths
// l = depth, depth - 1, depth - 2 (>= 2) of this tree: on level l the node
// size is its point count, above it the sum of the children's ranks, each
// rank estimated as min(size, K).  A node of size n, rank r and neighbour
// rows M costs (2/3)(n + r)^3 (pivot LU) + 2 n M (M + r) (Schur update).
int Tree::cost_depth(int K, std::vector<double>* costs) const {
  std::vector<std::vector<double>> pts_in((size_t)depth + 1);
  pts_in[depth].resize((size_t)levels[depth].n);
  for (int32_t i = 0; i < levels[depth].n; ++i)
    pts_in[depth][i] = (double)(levels[depth].pt_end[i] - levels[depth].pt_begin[i]);
  for (int l = depth - 1; l >= 2; --l) {
    const Level& L = levels[l];
    pts_in[l].assign((size_t)L.n, 0.0);
    for (int32_t i = 0; i < L.n; ++i)
      for (int e = L.child_ptr[i]; e < L.child_ptr[i + 1]; ++e) pts_in[l][i] += pts_in[l + 1][L.child[e]];
  }
  int best = depth;
  double best_cost = -1.0;
  if (costs) costs->clear();
  for (int cand = depth; cand >= std::max(2, depth - 2); --cand) {
    std::vector<double> nsz = pts_in[cand];
    double total = 0.0;
    for (int l = cand; l >= 2; --l) {
      const Level& L = levels[l];
      if (l < cand) {  // sizes from the children's estimated ranks
        const std::vector<double>& fine = nsz;
        std::vector<double> up((size_t)L.n, 0.0);
        for (int32_t i = 0; i < L.n; ++i)
          for (int e = L.child_ptr[i]; e < L.child_ptr[i + 1]; ++e) up[i] += std::min(fine[L.child[e]], (double)K);
        nsz.swap(up);
      }
      for (int32_t i = 0; i < L.n; ++i) {
        const double nv = nsz[i], rv = std::min(nv, (double)K);
        double Mv = 0.0;
        for (int e = L.nbr_ptr[i]; e < L.nbr_ptr[i + 1]; ++e) Mv += nsz[L.nbr[e]];
        total += 2.0 / 3.0 * (nv + rv) * (nv + rv) * (nv + rv) + 2.0 * nv * Mv * (Mv + rv);
      }
    }
    if (costs) costs->push_back(total);
    if (best_cost < 0.0 || total < best_cost) {
      best_cost = total;
      best = cand;
    }
  }
  return best;
}

std::string Tree::coincident(const double* pts) const {
  const Level& L = levels[depth];
  std::vector<int64_t> idx;
  for (int32_t b = 0; b < L.n; ++b) {
    idx.clear();
    for (int64_t t = L.pt_begin[b]; t < L.pt_end[b]; ++t) idx.push_back(perm[(size_t)t]);
    auto less = [&](int64_t a, int64_t c) {
      for (int e = 0; e < 3; ++e)
        if (pts[3 * a + e] != pts[3 * c + e]) return pts[3 * a + e] < pts[3 * c + e];
      return a < c;
    };
    std::sort(idx.begin(), idx.end(), less);
    for (size_t q = 1; q < idx.size(); ++q) {
      const int64_t a = idx[q - 1], c = idx[q];
      if (pts[3 * a] == pts[3 * c] && pts[3 * a + 1] == pts[3 * c + 1] && pts[3 * a + 2] == pts[3 * c + 2])
        return "points " + std::to_string(std::min(a, c)) + " and " + std::to_string(std::max(a, c)) +
               " coincide (the kernel 1/(4 pi r) is undefined at r = 0)";
    }
  }
  return "";
}

void Tree::box(int l, int32_t i, double c[3], double* half) const {
  const double side = 2.0 * H / (double)(1LL << l);
  const Level& L = levels[l];
  for (int e = 0; e < 3; ++e) c[e] = lo[e] + ((double)L.coord[3 * i + e] + 0.5) * side;
  *half = side / 2.0;
}

static void point_keys(const double* pts, int64_t n, const double lo[3], double H, int level,
                       std::vector<int32_t>& key) {
  const int64_t m = 1LL << level;
  const double s = (double)m / (2.0 * H);
  key.resize((size_t)(3 * n));
  for (int64_t p = 0; p < n; ++p)
    for (int e = 0; e < 3; ++e) {
      const double t = (pts[3 * p + e] - lo[e]) * s;
      double f = std::floor(t);
      if (f < 0.0) f = 0.0;
      if (f > (double)(m - 1)) f = (double)(m - 1);
      key[3 * p + e] = (int32_t)f;
    }
}

std::string Tree::build(const double* pts, int64_t n, int leaf_max, int sig, int depth_req, int tau, int colouring) {
  if (n < 1) return "need at least one point";
  if (leaf_max < 1) return "leaf_max must be positive";
  sigma = sig;
  double pmin[3], pmax[3];
  for (int e = 0; e < 3; ++e) {
    pmin[e] = pts[e];
    pmax[e] = pts[e];
  }
  for (int64_t p = 0; p < n; ++p)
    for (int e = 0; e < 3; ++e) {
      const double v = pts[3 * p + e];
      if (!std::isfinite(v)) return "non-finite coordinate";
      pmin[e] = std::min(pmin[e], v);
      pmax[e] = std::max(pmax[e], v);
    }
  double ext = 0.0;
  for (int e = 0; e < 3; ++e) ext = std::max(ext, pmax[e] - pmin[e]);
  H = ext / 2.0;
  if (!(H > 0.0)) return "all points coincide";
  for (int e = 0; e < 3; ++e) {
    const double centre = (pmin[e] + pmax[e]) / 2.0;
    lo[e] = centre - H;
  }
  // depth: smallest level >= 2 whose fullest leaf holds <= leaf_max points
  std::vector<int32_t> key;
  std::vector<int64_t> code((size_t)n);
  int L = depth_req >= 2 ? depth_req : 2;
  for (;; ++L) {
    if (L > 10) return "leaf size not reachable (too many coincident points)";
    if (depth_req >= 2) {  // the requested depth, whatever the leaf sizes
      point_keys(pts, n, lo, H, L, key);
      const int64_t m = 1LL << L;
      for (int64_t p = 0; p < n; ++p) code[p] = lex(key[3 * p], key[3 * p + 1], key[3 * p + 2], m);
      break;
    }
    point_keys(pts, n, lo, H, L, key);
    const int64_t m = 1LL << L;
    for (int64_t p = 0; p < n; ++p) code[p] = lex(key[3 * p], key[3 * p + 1], key[3 * p + 2], m);
    std::vector<int64_t> sorted(code);
    std::sort(sorted.begin(), sorted.end());
    int64_t best = 0;
    for (int64_t a = 0; a < n;) {
      int64_t b = a;
      while (b < n && sorted[b] == sorted[a]) ++b;
      best = std::max(best, b - a);
      a = b;
    }
    if (best <= leaf_max) break;
  }
  depth = L;
  perm.resize((size_t)n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return code[a] < code[b]; });
  levels.assign((size_t)L + 1, Level());
  // leaf level
  {
    Level& lv = levels[L];
    lv.level = L;
    for (int64_t t = 0; t < n;) {
      int64_t u = t;
      const int64_t c = code[perm[t]];
      while (u < n && code[perm[u]] == c) ++u;
      const int64_t p = perm[t];
      lv.coord.push_back(key[3 * p]);
      lv.coord.push_back(key[3 * p + 1]);
      lv.coord.push_back(key[3 * p + 2]);
      lv.pt_begin.push_back(t);
      lv.pt_end.push_back(u);
      t = u;
    }
    lv.n = (int32_t)lv.pt_begin.size();
  }
  // coarser levels by shifting coordinates
  for (int l = L - 1; l >= 2; --l) {
    const Level& f = levels[l + 1];
    Level& c = levels[l];
    c.level = l;
    const int64_t m = 1LL << l;
    std::vector<std::pair<int64_t, int32_t>> codes;
    codes.reserve(f.n);
    for (int32_t i = 0; i < f.n; ++i)
      codes.push_back({lex(f.coord[3 * i] >> 1, f.coord[3 * i + 1] >> 1, f.coord[3 * i + 2] >> 1, m), i});
    std::sort(codes.begin(), codes.end());
    for (size_t a = 0; a < codes.size(); ++a) {
      if (a > 0 && codes[a].first == codes[a - 1].first) continue;
      const int32_t i = codes[a].second;
      c.coord.push_back(f.coord[3 * i] >> 1);
      c.coord.push_back(f.coord[3 * i + 1] >> 1);
      c.coord.push_back(f.coord[3 * i + 2] >> 1);
    }
    c.n = (int32_t)(c.coord.size() / 3);
  }
  // parent / children and lists
  for (int l = 2; l <= L; ++l) {
    Level& lv = levels[l];
    const int64_t m = 1LL << l;
    std::unordered_map<int64_t, int32_t> index;
    index.reserve((size_t)lv.n * 2);
    for (int32_t i = 0; i < lv.n; ++i) index[lex(lv.coord[3 * i], lv.coord[3 * i + 1], lv.coord[3 * i + 2], m)] = i;
    auto find = [&](int i, int j, int k) -> int32_t {
      if (i < 0 || j < 0 || k < 0 || i >= m || j >= m || k >= m) return -1;
      auto it = index.find(lex(i, j, k, m));
      return it == index.end() ? -1 : it->second;
    };
    lv.parent.assign((size_t)lv.n, -1);
    if (l > 2) {
      const Level& pc = levels[l - 1];
      const int64_t mp = 1LL << (l - 1);
      std::unordered_map<int64_t, int32_t> pidx;
      pidx.reserve((size_t)pc.n * 2);
      for (int32_t i = 0; i < pc.n; ++i) pidx[lex(pc.coord[3 * i], pc.coord[3 * i + 1], pc.coord[3 * i + 2], mp)] = i;
      for (int32_t i = 0; i < lv.n; ++i)
        lv.parent[i] = pidx.at(lex(lv.coord[3 * i] >> 1, lv.coord[3 * i + 1] >> 1, lv.coord[3 * i + 2] >> 1, mp));
    }
    lv.nbr_ptr.assign(1, 0);
    lv.il_ptr.assign(1, 0);
    for (int32_t a = 0; a < lv.n; ++a) {
      const int x = lv.coord[3 * a], y = lv.coord[3 * a + 1], z = lv.coord[3 * a + 2];
      for (int dk = -1; dk <= 1; ++dk)
        for (int dj = -1; dj <= 1; ++dj)
          for (int di = -1; di <= 1; ++di) {
            if (!di && !dj && !dk) continue;
            const int32_t v = find(x + di, y + dj, z + dk);
            if (v >= 0) lv.nbr.push_back(v);
          }
      lv.nbr_ptr.push_back((int32_t)lv.nbr.size());
      // interaction list: children of the parent's neighbours (the whole
      // 6 x 6 x 6 block around the parent) at distance >= 2
      const int bx = 2 * (x >> 1) - 2, by = 2 * (y >> 1) - 2, bz = 2 * (z >> 1) - 2;
      for (int k = bz; k < bz + 6; ++k)
        for (int j = by; j < by + 6; ++j)
          for (int i = bx; i < bx + 6; ++i) {
            const int d = std::max(std::abs(i - x), std::max(std::abs(j - y), std::abs(k - z)));
            if (d < 2) continue;
            const int32_t v = find(i, j, k);
            if (v >= 0) lv.il.push_back(v);
          }
      lv.il_ptr.push_back((int32_t)lv.il.size());
    }
    // colouring (Alg. 3)
    std::vector<uint8_t> occ((size_t)(m * m * m), 0);
    for (int32_t i = 0; i < lv.n; ++i) occ[(size_t)lex(lv.coord[3 * i], lv.coord[3 * i + 1], lv.coord[3 * i + 2], m)] = 1;
    std::vector<int32_t> grid;
    if (l < tau) {  // one node per colour, in scan order
      grid.assign(occ.size(), -1);
      int32_t g = 0;
      for (size_t e = 0; e < occ.size(); ++e)
        if (occ[e]) grid[e] = g++;
      lv.ncolour = g;
    } else if (colouring == 1) {
      std::vector<int32_t> col;
      lv.ncolour = colour_lookback(lv, (int)m, sigma, col);
      grid.assign(occ.size(), -1);
      for (int32_t i = 0; i < lv.n; ++i)
        grid[(size_t)lex(lv.coord[3 * i], lv.coord[3 * i + 1], lv.coord[3 * i + 2], m)] = col[i];
    } else {
      lv.ncolour = colour_grid(occ, (int)m, sigma, grid);
    }
    lv.colour.resize((size_t)lv.n);
    std::vector<int32_t> cnt((size_t)lv.ncolour + 1, 0);
    for (int32_t i = 0; i < lv.n; ++i) {
      lv.colour[i] = grid[(size_t)lex(lv.coord[3 * i], lv.coord[3 * i + 1], lv.coord[3 * i + 2], m)];
      cnt[lv.colour[i] + 1]++;
    }
    for (int32_t c = 0; c < lv.ncolour; ++c) cnt[c + 1] += cnt[c];
    lv.grp_ptr = cnt;
    lv.grp.resize((size_t)lv.n);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t i = 0; i < lv.n; ++i) lv.grp[fill[lv.colour[i]]++] = i;
  }
  for (int l = 2; l < L; ++l) {
    Level& c = levels[l];
    const Level& f = levels[l + 1];
    std::vector<int32_t> cnt((size_t)c.n + 1, 0);
    for (int32_t i = 0; i < f.n; ++i) cnt[f.parent[i] + 1]++;
    for (int32_t i = 0; i < c.n; ++i) cnt[i + 1] += cnt[i];
    c.child_ptr = cnt;
    c.child.resize((size_t)f.n);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t i = 0; i < f.n; ++i) c.child[fill[f.parent[i]]++] = i;
  }
  return std::string();
}

}  // namespace ifmm
