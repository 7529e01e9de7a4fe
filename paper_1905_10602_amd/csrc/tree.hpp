// Host-side octree, neighbour / interaction lists and greedy colouring.
//
// Integer work only (apart from the box keys, which are single IEEE-754
// operations compiled without FMA contraction), so the structure is
// bit-reproducible.  Definitions follow Sec. 2.1 (neighbours, interaction
// list), the normalised distance equation of Sec. 3 and Alg. 3 (colouring).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ifmm {

struct Level {
  int level = 0;
  int32_t n = 0;                          // non-empty boxes, lexicographic (k, j, i)
  std::vector<int32_t> coord;             // 3 * n : (i, j, k) per node
  std::vector<int32_t> parent;            // index in level - 1, -1 at level 2
  std::vector<int32_t> child_ptr, child;  // CSR, children sorted by index
  std::vector<int32_t> nbr_ptr, nbr;      // CSR, N_i sorted
  std::vector<int32_t> il_ptr, il;        // CSR, I_i sorted
  std::vector<int32_t> colour;            // Alg. 3 colour per node
  int32_t ncolour = 0;
  std::vector<int32_t> grp_ptr, grp;      // CSR over colours, nodes ascending
  std::vector<int64_t> pt_begin, pt_end;  // leaf level only: ranges in tree order

  int dist(int32_t a, int32_t b) const;
};

struct Tree {
  int depth = 0;
  double lo[3] = {0, 0, 0};
  double H = 0;
  int sigma = 0;
  std::vector<int64_t> perm;   // perm[t] = original index of the t-th point in tree order
  std::vector<Level> levels;   // index = level; entries 0 and 1 unused

  // Builds everything; returns an empty string on success, else the reason.
  // depth_req: 0 = smallest level >= 2 with at most leaf_max points per leaf,
  // >= 2 = that level.  Levels below tau get one node per colour (scan order):
  // they are eliminated one node at a time (the matrix-parallel levels of
  // Sec. 4.2); the others are coloured by Alg. 3 (colouring = 0) or by the
  // look-back greedy (colouring = 1).
  std::string build(const double* pts, int64_t n, int leaf_max, int sigma, int depth_req = 0, int tau = 2,
                    int colouring = 0);
  // Box centre and half-side of node i at level l.
  void box(int l, int32_t i, double c[3], double* half) const;
  // After build(): an empty string if no two points coincide, else a message
  // naming one coincident pair by original index (the kernel is undefined at
  // r = 0).  Coincident points share a leaf, so each leaf is checked alone.
  std::string coincident(const double* pts) const;
  // The depth among depth, depth - 1, depth - 2 with the smallest estimated
  // factorisation cost (costs, if given, receives the estimates in that order).
  int cost_depth(int K, std::vector<double>* costs = nullptr) const;
};

// Alg. 3 on an m x m x m occupancy grid indexed [k][j][i]; returns the number
// of colours, colour[] = -1 for empty cells.
int32_t colour_grid(const std::vector<uint8_t>& occ, int m, int sigma, std::vector<int32_t>& colour);
// Look-back greedy colouring of the nodes of one level (colour per node).
int32_t colour_lookback(const Level& lv, int m, int sigma, std::vector<int32_t>& colour);

}  // namespace ifmm
