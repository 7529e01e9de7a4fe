// Black-box (Chebyshev) FMM matrix-vector product and the preconditioned
// GMRES of the FMBEM driver (Alg. 4 and 5): state and entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "tree.hpp"

namespace ifmm {

struct Handle;
struct BdHandle;

struct FmmHandle {
  Tree tree;
  int64_t N = 0;
  int nc = 5, K = 125, leaf_max = 64;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // host mirrors
  std::vector<int64_t> node_base;  // first global node index of each level
  int64_t nodes = 0;
  // M2L pair table: pairs grouped by (level, offset); GEMM tasks of <= 64 pairs
  int64_t npairs = 0;
  struct GemmTask {
    int32_t off, count;
    int64_t start;
  };
  std::vector<GemmTask> tasks;
  // device
  double *d_pts = nullptr, *d_w = nullptr, *d_diag = nullptr;  // tree order
  int64_t* d_perm = nullptr;
  int64_t* d_pt_begin = nullptr;                               // leaves, n_leaf + 1 entries
  int32_t *d_leaf_coord = nullptr, *d_nbr_ptr = nullptr, *d_nbr = nullptr;
  int32_t *d_node_oct = nullptr, *d_node_par = nullptr;        // global node index -> octant / parent (global)
  int32_t *d_child_ptr = nullptr, *d_child = nullptr;          // global CSR
  int64_t *d_tp_ptr = nullptr, *d_tp = nullptr;                // target (global) -> pair positions
  int32_t* d_pair_src = nullptr;                               // global source node per pair
  GemmTask* d_tasks = nullptr;
  double* d_half = nullptr;                                    // half-side per level
  int32_t* d_node_level = nullptr;
  double *d_S = nullptr, *d_m2m = nullptr, *d_m2l = nullptr;
  double *d_mult = nullptr, *d_loc = nullptr, *d_gath = nullptr, *d_part = nullptr;
  double *d_xs = nullptr, *d_ys = nullptr;
  // GMRES work space
  double* d_gm = nullptr;
  int64_t gm_bytes = 0;
  // statistics
  int64_t matvecs = 0;
  double t_matvec = 0, flops_m2l = 0;
};

int fmm_setup(FmmHandle& h, const double* pts, int64_t n, const double* w, const double* diag, double diag_scalar,
              std::string& err);
// y = A~ x for device vectors in the caller's point order (one column).
int fmm_apply(FmmHandle& h, const double* x, double* y, std::string& err);
// Right-preconditioned FGMRES(restart) from x = 0 on device vectors; pre may be null.
int fmm_gmres(FmmHandle& h, Handle* pre, const double* b, double* x, double tol, int restart, int maxit, int* iters,
              double* relres, std::string& err, BdHandle* bd = nullptr);
void fmm_release(FmmHandle& h);

}  // namespace ifmm
