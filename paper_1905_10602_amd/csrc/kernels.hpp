// HIP kernels of the IFMM factorisation and solve (gfx950, FP64).
//
// One workgroup (256 threads) per task: a node, a block, a neighbour row
// block or a changed basis.  Sizes come from the task tables, so batches of
// uneven nodes run in one launch per step and colour.
#pragma once

#include <hip/hip_runtime.h>

#include "cheb.hpp"
#include "dense.hpp"
#include "engine.hpp"

namespace ifmm {

// Static per-level structure as seen by the kernels.
struct LevelView {
  double* arena;
  const int32_t *n, *r, *rc, *coord;
  const int32_t *near_ptr, *near_idx, *il_ptr, *il_idx;
  const int64_t *near_off, *p2m_off, *l2p_off, *sig_off, *m2m_off, *l2l_off;
  double* const* il_blk;  // M2L block (t, il_idx[s]) of slot s; leading dimension ilcap[t]
  const int32_t* ilcap;
  const int64_t *cp2m_off, *cl2p_off, *T_off, *S_off;  // Chebyshev-basis operators and initial transforms
  const int32_t* chg;                                   // changed-node index per node (-1 = unchanged)
};

__device__ inline int dist3(const int32_t* coord, int a, int b) {
  int d = abs(coord[3 * a] - coord[3 * b]);
  d = max(d, abs(coord[3 * a + 1] - coord[3 * b + 1]));
  return max(d, abs(coord[3 * a + 2] - coord[3 * b + 2]));
}

// near block (p, q), dist(p, q) <= 1: offset in the arena (ld = n_p)
__device__ inline int64_t near_block(const LevelView& V, int p, int q) {
  for (int s = V.near_ptr[p]; s < V.near_ptr[p + 1]; ++s)
    if (V.near_idx[s] == q) return V.near_off[s];
  return -1;
}

// slot of the M2L block (t, s), s in I_t (binary search in the sorted list)
__device__ inline int il_slot(const LevelView& V, int t, int s) {
  int lo = V.il_ptr[t], hi = V.il_ptr[t + 1] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int v = V.il_idx[mid];
    if (v == s) return mid;
    if (v < s) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}


// Unit-side M2L for all 343 offsets d in [-3, 3]^3: U_d[m, m'] = K(d + xb_m / 2, xb_m' / 2).
__global__ void __launch_bounds__(NT) k_unit_m2l(int nc, double* out) {
  const int o = blockIdx.x;
  const int dx = o % 7 - 3, dy = (o / 7) % 7 - 3, dz = o / 49 - 3;
  const int K = nc * nc * nc;
  double* U = out + (int64_t)o * K * K;
  const bool near = abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1;
  if (K > 0) WG_FOR2(K, K, m, mp) {
    double v = 0.0;
    if (!near) {
      const double x = dx + 0.5 * (cheb_node(nc, m % nc) - cheb_node(nc, mp % nc));
      const double y = dy + 0.5 * (cheb_node(nc, (m / nc) % nc) - cheb_node(nc, (mp / nc) % nc));
      const double z = dz + 0.5 * (cheb_node(nc, m / (nc * nc)) - cheb_node(nc, mp / (nc * nc)));
      v = 1.0 / (4.0 * M_PI * sqrt(x * x + y * y + z * z));
    }
    U[m + (int64_t)mp * K] = v;
  }
}

// G_d = U_d^T U_d for every offset (source-side weight term).
__global__ void __launch_bounds__(NT) k_unit_gram(int K, const double* unit, double* uus) {
  const int o = blockIdx.x;
  wg_gemm(K, K, K, 1.0, unit + (int64_t)o * K * K, K, true, unit + (int64_t)o * K * K, K, false, 0.0,
          uus + (int64_t)o * K * K, K);
}

// M2M from a child in octant o (bit e set = upper half along axis e) to its parent.
__global__ void __launch_bounds__(NT) k_m2m8(int nc, double* out) {
  const int o = blockIdx.x;
  const int K = nc * nc * nc;
  double* M = out + (int64_t)o * K * K;
  const double sx = (o & 1) ? 0.5 : -0.5, sy = (o & 2) ? 0.5 : -0.5, sz = (o & 4) ? 0.5 : -0.5;
  if (K > 0) WG_FOR2(K, K, m, mp) {
    const double x = sx + 0.5 * cheb_node(nc, mp % nc);
    const double y = sy + 0.5 * cheb_node(nc, (mp / nc) % nc);
    const double z = sz + 0.5 * cheb_node(nc, mp / (nc * nc));
    M[m + (int64_t)mp * K] =
        cheb_S(nc, m % nc, x) * cheb_S(nc, (m / nc) % nc, y) * cheb_S(nc, m / (nc * nc), z);
  }
}

__device__ inline int octant_of(const int32_t* coord, int i) {
  return (coord[3 * i] & 1) | ((coord[3 * i + 1] & 1) << 1) | ((coord[3 * i + 2] & 1) << 2);
}

__device__ inline int offset_index(const int32_t* coord, int t, int s) {
  const int dx = coord[3 * t] - coord[3 * s], dy = coord[3 * t + 1] - coord[3 * s + 1],
            dz = coord[3 * t + 2] - coord[3 * s + 2];
  return (dx + 3) + 7 * ((dy + 3) + 7 * (dz + 3));
}

// Far-field weight of every node of a level (top-down):
//   G_i = (1/L^2) sum_{l in I_i} U_{c_l - c_i}^T U_{c_l - c_i} + M2M_i^T G_parent M2M_i.
// The Laplace kernel is symmetric, so the target weight equals G_i.
__global__ void __launch_bounds__(NT) k_weights(int K, int nn, const int32_t* coord, const int32_t* il_ptr, const int32_t* il_idx,
                          const int32_t* parent, const double* uus, const double* m2m8, double invL2,
                          const double* Gpar, double* G, double* tmp) {
  const int i = blockIdx.x;
  double* Gi = G + (int64_t)i * K * K;
  for (int e = threadIdx.x; e < K * K; e += NT) {
    double acc = 0.0;
    for (int s = il_ptr[i]; s < il_ptr[i + 1]; ++s)
      acc += uus[(int64_t)offset_index(coord, il_idx[s], i) * K * K + e];
    Gi[e] = acc * invL2;
  }
  __syncthreads();
  if (Gpar) {
    const double* M = m2m8 + (int64_t)octant_of(coord, i) * K * K;
    const double* Gp = Gpar + (int64_t)parent[i] * K * K;
    double* t = tmp + (int64_t)i * K * K;
    wg_gemm(K, K, K, 1.0, Gp, K, false, M, K, false, 0.0, t, K);
    wg_gemm(K, K, K, 1.0, M, K, true, t, K, false, 1.0, Gi, K);
  }
}

// Leaf Chebyshev operators: P2Mc (K x n, ld K) and L2Pc (n x K, ld n).
__global__ void __launch_bounds__(NT) k_leaf_cheb(LevelView V, int nc, const double* pts, const double* w, const int64_t* pt_begin,
                            const double* lo, double side) {
  const int i = blockIdx.x;
  const int K = nc * nc * nc;
  const int n = V.n[i];
  double* P2M = V.arena + V.cp2m_off[i];
  double* L2P = V.arena + V.cl2p_off[i];
  const double h = 0.5 * side;
  double c[3];
  for (int e = 0; e < 3; ++e) c[e] = lo[e] + ((double)V.coord[3 * i + e] + 0.5) * side;
  const int64_t b = pt_begin[i];
  if (K > 0) WG_FOR2(K, n, m, j) {
    const double* p = pts + 3 * (b + j);
    const double s = cheb_S(nc, m % nc, (p[0] - c[0]) / h) * cheb_S(nc, (m / nc) % nc, (p[1] - c[1]) / h) *
                     cheb_S(nc, m / (nc * nc), (p[2] - c[2]) / h);
    P2M[m + (int64_t)j * K] = s * w[b + j];
    L2P[j + (int64_t)m * n] = s;
  }
}

// Near-field blocks of the leaves: P2P_pq[a, b] = K(x_a, x_b) w_b, diag on the self block.
__global__ void __launch_bounds__(NT) k_p2p(LevelView V, const int32_t* slot_row, const double* pts, const double* w,
                      const double* diag, const int64_t* pt_begin) {
  const int s = blockIdx.x;
  const int p = slot_row[s], q = V.near_idx[s];
  const int np = V.n[p], nq = V.n[q];
  double* B = V.arena + V.near_off[s];
  const int64_t bp = pt_begin[p], bq = pt_begin[q];
  if (np > 0) WG_FOR2(np, nq, a, bb) {
    double v;
    if (p == q && a == bb) {
      v = diag[bp + a];
    } else {
      const double* x = pts + 3 * (bp + a);
      const double* y = pts + 3 * (bq + bb);
      const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
      v = w[bq + bb] / (4.0 * M_PI * sqrt(dx * dx + dy * dy + dz * dz));
    }
    B[a + (int64_t)bb * np] = v;
  }
}

// Initial rank reduction, Gram step: Gs = P2Mc^T G P2Mc, Gt = L2Pc G L2Pc^T (n x n).
__global__ void __launch_bounds__(NT) k_reduce_gram(LevelView V, int K, const double* G, double* work, const int64_t* work_off) {
  const int i = blockIdx.x;
  const int n = V.n[i];
  if (n == 0) return;
  double* base = work + work_off[i];
  double* gs = base;
  double* gt = gs + (int64_t)n * n;
  double* t = gt + (int64_t)n * n;  // K x n
  const double* Gi = G + (int64_t)i * K * K;
  const double* P2M = V.arena + V.cp2m_off[i];
  const double* L2P = V.arena + V.cl2p_off[i];
  wg_gemm(K, n, K, 1.0, Gi, K, false, P2M, K, false, 0.0, t, K);
  wg_gemm(n, n, K, 1.0, P2M, K, true, t, K, false, 0.0, gs, n);
  wg_gemm(K, n, K, 1.0, Gi, K, false, L2P, n, true, 0.0, t, K);
  wg_gemm(n, n, K, 1.0, L2P, n, false, t, K, false, 0.0, gt, n);
}

// Batched symmetric eigen-decomposition in two launches around the host's
// rank decision: values (tridiagonalisation + bisection; cnt[t] = #{k :
// lam_k > eps2 * lam_0}) and then the k leading vectors.
struct EigTask {
  double *A, *V, *W, *lam, *IW;  // A n x n (destroyed), V n x k, W 3n, lam n, IW 5 n k
  int32_t n, k;
};
__device__ inline void eig_count(const EigTask& t, double eps2, int32_t* cnt) {
  if (threadIdx.x == 0) {
    const double l0 = t.lam[0];
    int c = 0;
    if (l0 > 0.0)
      for (int k = 0; k < t.n; ++k)
        if (t.lam[k] > eps2 * l0) ++c;
    cnt[blockIdx.x] = c;
  }
}

// cyclic Jacobi alternative (all vectors at once; W holds n x n)
__global__ void __launch_bounds__(NT) k_eig_jacobi(const EigTask* tasks, double eps2, int32_t* cnt) {
  const EigTask t = tasks[blockIdx.x];
  if (t.n == 0) {
    if (threadIdx.x == 0) cnt[blockIdx.x] = 0;
    return;
  }
  wg_syev_jacobi(t.n, t.A, t.n, t.V, t.n, t.W, t.lam);
  eig_count(t, eps2, cnt);
}

// big > 0: matrices of order >= big are left to the multi-workgroup reduction
__global__ void __launch_bounds__(NT) k_eig_values(const EigTask* tasks, double eps2, int32_t* cnt, int big) {
  const EigTask t = tasks[blockIdx.x];
  if (big > 0 && t.n >= big) return;
  if (t.n == 0) {
    if (threadIdx.x == 0) cnt[blockIdx.x] = 0;
    return;
  }
  wg_syev_values(t.n, t.A, t.n, t.W, t.lam);
  if (threadIdx.x == 0) {
    const double l0 = t.lam[0];
    int c = 0;
    if (l0 > 0.0)
      for (int k = 0; k < t.n; ++k)
        if (t.lam[k] > eps2 * l0) ++c;
    cnt[blockIdx.x] = c;
  }
}

// Whether task (n, k) leaves its back-transform to k_ev_mask / k_ev_apply
// (big > 0: orders from big on, with at least one full block of reflectors).
__device__ inline bool ev_split(int n, int k, int big) { return big > 0 && n >= big && n >= 34 && k > 0; }

__global__ void __launch_bounds__(NT) k_eig_vectors(const EigTask* tasks, int big) {
  const EigTask t = tasks[blockIdx.x];
  if (t.n == 0 || t.k == 0) return;
  wg_syev_vectors(t.n, t.A, t.n, t.W, t.lam, t.k, t.V, t.n, t.IW, !ev_split(t.n, t.k, big));
}

// Blocked back-transform of the large tasks, many workgroups per matrix.
// The reflectors v_q (unit vectors, rows q+1.. of column q of A) are applied
// 32 at a time in compact WY form, H_b0 ... H_b1-1 = I - V T V^T, where
// T^-1 = diag(1/2) + (strict upper part of V^T V) for H_q = I - 2 v_q v_q^T
// (Joffrain, Low, Quintana-Orti, van de Geijn and van Zee, "Accumulating
// Householder transformations, revisited", 2006).  k_ev_mask first zeroes
// what V must read as zero: column q on and above the diagonal, and the whole
// column of a skipped reflector (tau_q = 0).  grid (ceil(n_max / 64), task).
__global__ void __launch_bounds__(NT) k_ev_mask(const EigTask* tasks, int big) {
  const EigTask t = tasks[blockIdx.y];
  const int n = t.n;
  if (!ev_split(n, t.k, big)) return;
  const int q0 = blockIdx.x * 64, q1 = min(n - 2, q0 + 64);
  const double* tau = t.W + 2 * n;
  for (int q = q0; q < q1; ++q) {
    const int rend = tau[q] != 0.0 ? q + 1 : n;
    for (int r = threadIdx.x; r < rend; r += NT) t.A[r + (int64_t)q * n] = 0.0;
  }
}

// X <- H_0 ... H_{n-3} X on a block of 64 columns of X (grid (ceil(k_max /
// 64), task)), reflector blocks from the last to the first: with the rows
// b0+1.. of the block's columns, G = V^T V and B = V^T X, then T^-1 W = B by
// back substitution (W = T B) and X -= V W.
__global__ void __launch_bounds__(NT) k_ev_apply(const EigTask* tasks, int big) {
  __shared__ double sG[32 * 32], sB[32 * 64];
  const EigTask t = tasks[blockIdx.y];
  const int n = t.n, k = t.k;
  if (!ev_split(n, k, big)) return;
  const int c0 = blockIdx.x * 64;
  if (c0 >= k) return;
  const int kc = min(64, k - c0);
  double* X = t.V + (int64_t)c0 * n;
  for (int b1 = n - 2; b1 > 0; b1 -= 32) {
    const int b0 = max(0, b1 - 32), nb = b1 - b0, mb = n - b0 - 1;
    const double* Vs = t.A + (b0 + 1) + (int64_t)b0 * n;
    double* Xs = X + (b0 + 1);
    wg_gemm<false>(nb, nb, mb, 1.0, Vs, n, true, Vs, n, false, 0.0, sG, 32);
    wg_gemm<false>(nb, kc, mb, 1.0, Vs, n, true, Xs, n, false, 0.0, sB, 32);
    for (int j = threadIdx.x; j < kc; j += NT)
      for (int q = nb - 1; q >= 0; --q) {
        double acc = sB[q + 32 * j];
        for (int p = q + 1; p < nb; ++p) acc -= sG[q + 32 * p] * sB[p + 32 * j];
        sB[q + 32 * j] = 2.0 * acc;
      }
    __syncthreads();
    wg_gemm<false>(mb, kc, nb, -1.0, Vs, n, false, sB, 32, false, 1.0, Xs, n);
  }
}

// ---- Householder tridiagonalisation spread over many workgroups (large
// matrices, batched over the matrices of a colour).  The same reduction as
// wg_syev_values, one reflector per step: a one-workgroup step kernel per
// matrix (reduce p = S v from partial sums, K = p^T v, w = p - K v, update the
// leading column of S, form the next reflector from it) and a tiled kernel
// over the trailing matrix (S -= 2 (v w^T + w v^T) on 64 x 64 tiles, each
// tile also accumulating its part of the next product S' v').  Per step the
// trailing matrix is read and written once by the whole device instead of
// by one compute unit.
struct TrdTask {
  double* A;     // n x n, ld n: symmetric input, overwritten (reflectors below the subdiagonal)
  double* W;     // d (n), e (n), tau (n), as the one-workgroup solver leaves them
  double* vec;   // 3 n: v, w of the current step and the next reflector, in trailing coordinates
  double* part;  // n x ceil(n / 64): partial sums of the next product, one column per column tile
  int32_t n, slot;  // order; index of the matrix in the caller's EigTask table and count array
};

// Householder vector of x (length m, in place in A's column): sets e / tau of
// step `k`; returns the vector (normalised, 0 if x[1:] is already zero) in v.
__device__ inline void trd_reflector(double* x, int m, double* e, double* tau, int k, double* v) {
  const int tid = threadIdx.x;
  double part = 0.0;
  for (int i = 1 + tid; i < m; i += NT) part += x[i] * x[i];
  const double sig = wg_sum(part);
  __syncthreads();
  const double x0 = x[0];
  if (sig == 0.0) {
    for (int i = tid; i < m; i += NT) v[i] = 0.0;
    if (tid == 0) { e[k] = x0; tau[k] = 0.0; }
    __syncthreads();
    return;
  }
  const double alpha = -copysign(sqrt(x0 * x0 + sig), x0);
  const double v0 = x0 - alpha;
  const double inv = 1.0 / sqrt(sig + v0 * v0);
  for (int i = tid; i < m; i += NT) v[i] = (i == 0 ? v0 : x[i]) * inv;
  __syncthreads();
  for (int i = tid; i < m; i += NT) x[i] = v[i];
  if (tid == 0) { e[k] = alpha; tau[k] = 1.0; }
  __syncthreads();
}

// Start: the first reflector (from column 0) into vec's next-reflector slot;
// v, w of the "previous step" are zero, so the first tiled pass only forms S v.
__global__ void __launch_bounds__(NT) k_trd_start(const TrdTask* tasks) {
  const TrdTask t = tasks[blockIdx.x];
  const int n = t.n;
  if (n < 3) return;
  const int m = n - 1;
  double* v = t.vec;
  double* w = t.vec + n;
  double* vn = t.vec + 2 * n;
  for (int i = threadIdx.x; i < m; i += NT) { v[i] = 0.0; w[i] = 0.0; }
  trd_reflector(t.A + 1, m, t.W + n, t.W + 2 * n, 0, vn);
}

// Tiled pass after step k (k = -1: the first product only) over the lower
// triangle of the trailing matrix S = A[k+2:, k+2:] (order m = n - k - 2; the
// upper triangle is never read): S -= 2 (v w^T + w v^T) with the step's v, w
// (already in S's coordinates), and the partial sums of p = S vn with S
// symmetric.  A tile (ti >= tj) contributes S_tile vn_J to the rows of block
// ti (slot tj of part) and S_tile^T vn_I to the rows of block tj (slot ti),
// so every (row, slot) is written by exactly one tile; a diagonal tile adds
// both into slot ti.  grid (lower tiles of the largest S, task).
// Thread (tx, ty) = (tid % 16, tid / 16) owns rows I + tx + 16a and columns
// J + ty + 16b (a, b < 4): its 16 loads are issued together (16 lanes read
// 128 contiguous bytes of a column), and the row and column sums meet in LDS.
__global__ void __launch_bounds__(NT) k_trd_tiles(const TrdTask* tasks, int k) {
  __shared__ double rowp[16][64], colp[16][64];
  const TrdTask t = tasks[blockIdx.y];
  const int n = t.n, m = n - k - 2;
  if (n < 3 || k > n - 3 || m <= 0) return;
  const int nb = (m + 63) / 64;
  const int tile = blockIdx.x;
  if (tile >= nb * (nb + 1) / 2) return;
  int ti = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) / 2 > tile) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
  const int tj = tile - ti * (ti + 1) / 2;
  const bool diag = ti == tj;
  const int I = 64 * ti, J = 64 * tj;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const auto v = gmem(t.vec);
  const auto w = gmem(t.vec + n);
  const auto vn = gmem(t.vec + 2 * n);
  const auto S = gmem(t.A + (k + 2) + (int64_t)(k + 2) * n);
  double vr[4], wr[4], vnr[4], vc[4], wc[4], vnc[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = I + tx + 16 * a, j = J + ty + 16 * a;
    vr[a] = i < m ? v[i] : 0.0;
    wr[a] = i < m ? w[i] : 0.0;
    vnr[a] = i < m ? vn[i] : 0.0;
    vc[a] = j < m ? v[j] : 0.0;
    wc[a] = j < m ? w[j] : 0.0;
    vnc[a] = j < m ? vn[j] : 0.0;
  }
  double x[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = I + tx + 16 * a, j = J + ty + 16 * b;
      x[a][b] = (i < m && j < m && (!diag || i >= j)) ? S[i + (int64_t)j * n] : 0.0;
    }
  double racc[4] = {0.0, 0.0, 0.0, 0.0}, cacc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = I + tx + 16 * a, j = J + ty + 16 * b;
      if (i < m && j < m && (!diag || i >= j)) {
        const double sv = x[a][b] - 2.0 * (vr[a] * wc[b] + wr[a] * vc[b]);
        x[a][b] = sv;
        racc[a] += sv * vnc[b];
        if (!diag || i > j) cacc[b] += sv * vnr[a];
      }
    }
  // the stores after every result (a wait for a load after a store would
  // also wait for the store)
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = I + tx + 16 * a, j = J + ty + 16 * b;
      if (i < m && j < m && (!diag || i >= j)) S[i + (int64_t)j * n] = x[a][b];
    }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    rowp[ty][tx + 16 * a] = racc[a];
    colp[tx][ty + 16 * a] = cacc[a];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    double r = 0.0, c = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      r += rowp[q][l];
      c += colp[q][l];
    }
    if (diag) {
      if (I + l < m) t.part[(int64_t)ti * n + I + l] = r + c;
    } else {
      if (I + l < m) t.part[(int64_t)tj * n + I + l] = r;
      if (J + l < m) t.part[(int64_t)ti * n + J + l] = c;
    }
  }
}

// Step k (0 <= k <= n - 3): p = sum of the partial sums (S_k v_k, S_k =
// A[k+1:, k+1:] of order m = n - k - 1), K = p^T v, w = p - K v, update of
// S_k's leading column, the next reflector from it, and v, w, vn of the
// following tiled pass in the coordinates of A[k+2:, k+2:].
__global__ void __launch_bounds__(NT) k_trd_step(const TrdTask* tasks, int k) {
  __shared__ double sp[TRD_MAXN], sv[TRD_MAXN], sw[TRD_MAXN];
  const TrdTask t = tasks[blockIdx.x];
  const int n = t.n;
  if (n < 3 || k > n - 3) return;
  const int m = n - k - 1, nb = (m + 63) / 64;
  const int tid = threadIdx.x;
  double* vec_v = t.vec;
  double* vec_w = t.vec + n;
  double* vec_n = t.vec + 2 * n;
  double* col = t.A + (k + 1) + (int64_t)k * n;  // reflector v_k, stored by the previous step
  for (int i = tid; i < m; i += NT) {
    double a = 0.0;
#pragma unroll 8
    for (int c = 0; c < nb; ++c) a += t.part[(int64_t)c * n + i];
    sp[i] = a;
    sv[i] = t.W[2 * n + k] != 0.0 ? col[i] : 0.0;  // tau_k = 0: no reflector at this step
  }
  __syncthreads();
  double kp = 0.0;
  for (int i = tid; i < m; i += NT) kp += sp[i] * sv[i];
  const double K = wg_sum(kp);
  for (int i = tid; i < m; i += NT) sw[i] = sp[i] - K * sv[i];
  __syncthreads();
  // leading column of S_k: column k + 1 of A, rows k + 1 ..
  double* S0 = t.A + (k + 1) + (int64_t)(k + 1) * n;
  for (int i = tid; i < m; i += NT) S0[i] -= 2.0 * (sv[i] * sw[0] + sw[i] * sv[0]);
  __syncthreads();
  const int m2 = m - 1;
  for (int i = tid; i < m2; i += NT) {
    vec_v[i] = sv[i + 1];
    vec_w[i] = sw[i + 1];
  }
  if (k + 3 < n) {
    trd_reflector(S0 + 1, m2, t.W + n, t.W + 2 * n, k + 1, sp);  // sp now holds the next reflector
    for (int i = tid; i < m2; i += NT) vec_n[i] = sp[i];
  } else {
    for (int i = tid; i < m2; i += NT) vec_n[i] = 0.0;
  }
}

// After the last step: the eigenvalues of the tridiagonal matrix by bisection
// on Sturm counts, spread over workgroups of NT eigenvalues each (grid
// (ceil(n_max / NT), task)).  Every workgroup stages d and e in LDS (the
// counts read them n times per bisection step) and forms the Gershgorin
// interval itself; workgroup 0 also stores d and the last off-diagonal in W.
// The values are those of the one-workgroup bisection, bit for bit (same
// interval, same steps; min and max reductions are exact).
__global__ void __launch_bounds__(NT) k_trd_bisect(const TrdTask* tasks, const EigTask* et) {
  __shared__ double sd[TRD_MAXN], se[TRD_MAXN];
  __shared__ double s_lo[NT / 64], s_hi[NT / 64];
  const TrdTask t = tasks[blockIdx.y];
  const int n = t.n, j0 = blockIdx.x * NT, tid = threadIdx.x;
  if (n < 3 || j0 >= n) return;
  double* lam = et[t.slot].lam;
  double* d = t.W;
  double* e = t.W + n;
  const double e_last = t.A[(n - 1) + (int64_t)(n - 2) * n];
  for (int i = tid; i < n; i += NT) {
    const double di = t.A[i + (int64_t)i * n];
    sd[i] = di;
    if (blockIdx.x == 0) d[i] = di;
    if (i + 1 < n) se[i] = i == n - 2 ? e_last : e[i];
  }
  if (blockIdx.x == 0 && tid == 0) e[n - 2] = e_last;
  __syncthreads();
  double lo = 0.0, hi = 0.0;
  bool any = false;
  for (int i = tid; i < n; i += NT) {
    const double rad = (i > 0 ? fabs(se[i - 1]) : 0.0) + (i + 1 < n ? fabs(se[i]) : 0.0);
    const double a = sd[i] - rad, b = sd[i] + rad;
    if (!any || a < lo) lo = a;
    if (!any || b > hi) hi = b;
    any = true;
  }
  if (!any) { lo = INFINITY; hi = -INFINITY; }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
  }
  if ((tid & 63) == 0) { s_lo[tid >> 6] = lo; s_hi[tid >> 6] = hi; }
  __syncthreads();
  lo = s_lo[0];
  hi = s_hi[0];
  for (int w = 1; w < NT / 64; ++w) { lo = fmin(lo, s_lo[w]); hi = fmax(hi, s_hi[w]); }
  const double nrm = fmax(fabs(lo), fabs(hi));
  const double tiny = 2.2e-16 * nrm + 1e-300;
  const int j = j0 + tid;
  if (j < n) {
    const int target = n - 1 - j;  // the j-th largest has n-1-j eigenvalues below it
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (a + b);
      if (b - a <= 4.4e-16 * nrm || mid <= a || mid >= b) break;
      if (sturm_count(n, sd, se, mid, tiny) > target) b = mid;
      else a = mid;
    }
    lam[j] = 0.5 * (a + b);
  }
}

// Count of eigenvalues above eps2 * lam_0 per task (one workgroup each); the
// tiny orders the reduction leaves untouched (n < 3) are solved here whole.
__global__ void __launch_bounds__(NT) k_trd_count(const TrdTask* tasks, const EigTask* et, double eps2, int32_t* cnt) {
  const TrdTask t = tasks[blockIdx.x];
  const EigTask e = et[t.slot];
  if (t.n == 0) {
    if (threadIdx.x == 0) cnt[t.slot] = 0;
    return;
  }
  if (t.n < 3) wg_syev_values(t.n, t.A, t.n, t.W, e.lam);
  const double l0 = e.lam[0];
  double c = 0.0;
  if (l0 > 0.0)
    for (int q = threadIdx.x; q < t.n; q += NT) c += e.lam[q] > eps2 * l0 ? 1.0 : 0.0;
  c = wg_sum(c);
  if (threadIdx.x == 0) cnt[t.slot] = (int32_t)c;
}

// ------------------------------------------------------------------ batched tiled GEMM
// C = alpha op(A) op(B) + beta C for many independent problems; grid
// (row tiles, column tiles, task), one 64 x 64 output tile per workgroup.
struct GemmTask {
  const double* A;
  const double* B;
  double* C;
  int32_t m, n, k, lda, ldb, ldc, tA, tB;
  double alpha, beta;
};
// mf: the FP64 matrix-core tile (every task of the launch with tB == 0).
template <bool mf>
__global__ void __launch_bounds__(NT) k_gemm_batch(const GemmTask* tasks) {
  const GemmTask t = tasks[blockIdx.z];
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  if (i0 >= t.m || j0 >= t.n) return;
  const int mm = min(64, t.m - i0), nn = min(64, t.n - j0);
  const double* Ab = t.tA ? t.A + (int64_t)i0 * t.lda : t.A + i0;
  const double* Bb = t.tB ? t.B + j0 : t.B + (int64_t)j0 * t.ldb;
  if constexpr (mf)
    wg_gemm_f64m(mm, nn, t.k, t.alpha, Ab, t.lda, Bb, t.ldb, t.beta, t.C + i0 + (int64_t)j0 * t.ldc, t.ldc,
                 t.tA != 0);
  else
    wg_gemm(mm, nn, t.k, t.alpha, Ab, t.lda, t.tA != 0, Bb, t.ldb, t.tB != 0, t.beta,
            t.C + i0 + (int64_t)j0 * t.ldc, t.ldc);
}

// ------------------------------------------------------------------ sketched recompression
// Randomised range finder on a Gram matrix G (n x n, PSD) with s columns
// (the predicted rank plus oversampling): Y = G Omega, Q = orth(Y),
// B = Q^T G Q, eigen-pairs of B (Rayleigh-Ritz).  Every direction outside
// span(Q) carries at most trace(G) - trace(B) of G's eigenvalue mass, so the
// sketch is accepted when that tail is <= eps^2 lambda_1 (no eigenvalue
// above the truncation threshold was missed) and fewer than s Ritz values
// pass the threshold; otherwise the full eigen-decomposition runs.
struct SkTask {
  const double* G;  // n x n
  double *O, *Y;    // O: Omega (R x s), later G Q (n x s);  Y (n x s), then Q
  double* B;        // s x s
  double* tr;       // trace(G), trace(B)
  int32_t n, s, R, chg;  // R = rows of the stacked factor W (G = W^T W); changed-node index
  uint32_t seed, side;
};

__device__ inline double sk_uniform(uint32_t seed, uint64_t idx) {
  uint64_t z = ((uint64_t)seed << 40) ^ (idx + 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;  // [-1, 1)
}

__global__ void __launch_bounds__(NT) k_sk_omega(const SkTask* tasks) {
  const SkTask t = tasks[blockIdx.y];
  const int64_t tot = (int64_t)t.R * t.s;
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * NT)
    t.O[e] = sk_uniform(t.seed, (uint64_t)e);
}

// Range sample of the stacked factor instead of the Gram matrix itself, so the
// sampled directions carry singular values, not their squares:
//   side 0:  Y = W^T Omega,  W = [diag(sig_s) P2M ; F_qp ...]   (rows: r, then m_q each)
//   side 1:  Y = W Omega,    W = [L2P diag(sig_t) , F_pq ...]   (columns likewise)
// grid (row tiles of n, column tiles of s, sketch task).  F32: the products
// on FP32 matrix cores (mixed form); the Rayleigh-Ritz step and the
// a-posteriori test that judge the sample stay FP64.
template <bool F32>
__global__ void __launch_bounds__(NT) k_sk_range(const Changed* chg, const FarRef* refs, const FarPair* far, const ElimNbr* nbrs,
                           const ElimRec* recs, const SkTask* tasks) {
  const SkTask t = tasks[blockIdx.z];
  const int I = blockIdx.x * 64, J = blockIdx.y * 64;
  if (I >= t.n || J >= t.s) return;
  const Changed C = chg[t.chg];
  const int n = C.n, r = C.r, s = t.s;
  const int mi = min(64, n - I), sj = min(64, s - J);
  const ElimRec R = recs[C.rec];
  const double* tb = C.tmp + (int64_t)t.side * r * n;  // scaled bases from k_gram_prep
  double* Y = t.Y + I + (int64_t)J * n;
  const double* Om = t.O + (int64_t)J * t.R;
  if (t.side == 0) {
    wg_gemm_p(F32, mi, sj, r, 1.0, tb + (int64_t)I * r, r, true, Om, t.R, false, 0.0, Y, n);
    int off = r;
    for (int k = 0; k < C.far_count; ++k) {
      const FarPair Pq = far[refs[C.far_begin + k].ba];
      const int mq = nbrs[R.nb_begin + Pq.a].m;
      wg_gemm_p(F32, mi, sj, mq, 1.0, Pq.F + (int64_t)I * mq, mq, true, Om + off, t.R, false, 1.0, Y, n);
      off += mq;
    }
  } else {
    wg_gemm_p(F32, mi, sj, r, 1.0, tb + I, n, false, Om, t.R, false, 0.0, Y, n);
    int off = r;
    for (int k = 0; k < C.far_count; ++k) {
      const FarPair Pq = far[refs[C.far_begin + k].ab];
      const int mq = nbrs[R.nb_begin + Pq.b].m;
      wg_gemm_p(F32, mi, sj, mq, 1.0, Pq.F + I, n, false, Om + off, t.R, false, 1.0, Y, n);
      off += mq;
    }
  }
}

// Column-by-column Gram-Schmidt with one reorthogonalisation pass; a column
// whose norm collapses below `drop` times its original norm only adds
// directions with singular values far below the truncation threshold and is
// set to zero (keeping Q orthonormal).  One workgroup per task.
__global__ void __launch_bounds__(NT) k_sk_orth(const SkTask* tasks, double drop) {
  __shared__ double s_c[NT];
  const SkTask t = tasks[blockIdx.x];
  const int n = t.n, k = t.s;
  double* X = t.Y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int j = 0; j < k; ++j) {
    double* xj = X + (int64_t)j * n;
    double part = 0.0;
    for (int r = tid; r < n; r += NT) part += xj[r] * xj[r];
    const double n0 = sqrt(wg_sum(part));
    for (int pass = 0; pass < 2; ++pass) {
      for (int i0 = 0; i0 < j; i0 += NT) {
        const int cnt = min(NT, j - i0);
        for (int i = i0 + wave; i < i0 + cnt; i += NT / 64) {
          const double* xi = X + (int64_t)i * n;
          double c = 0.0;
          for (int r = lane; r < n; r += 64) c += xi[r] * xj[r];
          for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
          if (lane == 0) s_c[i - i0] = c;
        }
        __syncthreads();
        for (int r = tid; r < n; r += NT) {
          double v = xj[r];
          for (int i = 0; i < cnt; ++i) v -= s_c[i] * X[r + (int64_t)(i0 + i) * n];
          xj[r] = v;
        }
        __syncthreads();
      }
    }
    part = 0.0;
    for (int r = tid; r < n; r += NT) part += xj[r] * xj[r];
    const double n2 = sqrt(wg_sum(part));
    const double sc = (n2 > drop * n0 && n2 > 0.0) ? 1.0 / n2 : 0.0;
    for (int r = tid; r < n; r += NT) xj[r] *= sc;
    __syncthreads();
  }
}

// Top singular values of an 8-column range sample Y (n x 8): sqrt of the
// eigenvalues of Y^T Y (cyclic Jacobi on the 8 x 8 matrix), descending.
// These are the "sketched singular values" fed to the rank predictor.
__global__ void __launch_bounds__(NT) k_feat_sv(const SkTask* tasks, double* out) {
  __shared__ double g[8][8];
  const SkTask t = tasks[blockIdx.x];
  const int n = t.n;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int pr = wave; pr < 64; pr += NT / 64) {
    const int a = pr >> 3, b = pr & 7;
    double c = 0.0;
    if (a <= b)
      for (int r = lane; r < n; r += 64) c += t.Y[r + (int64_t)a * n] * t.Y[r + (int64_t)b * n];
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0 && a <= b) {
      g[a][b] = c;
      g[b][a] = c;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int sweep = 0; sweep < 30; ++sweep) {
      double off = 0.0;
      for (int p = 0; p < 8; ++p)
        for (int q = p + 1; q < 8; ++q) off += g[p][q] * g[p][q];
      if (off == 0.0) break;
      for (int p = 0; p < 8; ++p)
        for (int q = p + 1; q < 8; ++q) {
          if (g[p][q] == 0.0) continue;
          const double th = (g[q][q] - g[p][p]) / (2.0 * g[p][q]);
          const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          const double cs = 1.0 / sqrt(tt * tt + 1.0), sn = tt * cs;
          for (int k = 0; k < 8; ++k) {
            const double gp = g[k][p], gq = g[k][q];
            g[k][p] = cs * gp - sn * gq;
            g[k][q] = sn * gp + cs * gq;
          }
          for (int k = 0; k < 8; ++k) {
            const double gp = g[p][k], gq = g[q][k];
            g[p][k] = cs * gp - sn * gq;
            g[q][k] = sn * gp + cs * gq;
          }
        }
    }
    double ev[8];
    for (int k = 0; k < 8; ++k) ev[k] = fmax(g[k][k], 0.0);
    for (int a = 0; a < 8; ++a)
      for (int b = a + 1; b < 8; ++b)
        if (ev[b] > ev[a]) {
          const double x = ev[a];
          ev[a] = ev[b];
          ev[b] = x;
        }
    for (int k = 0; k < 8; ++k) out[8 * blockIdx.x + k] = sqrt(ev[k]);
  }
}

// Blocked classical Gram-Schmidt with reorthogonalisation (BCGS2) of the
// range sample, 64 columns per block: the projections against the earlier
// blocks are batched GEMMs on many workgroups (k_gemm_batch); these two
// kernels give the column norms before any projection and orthonormalise the
// columns inside a block (same dependence rule as k_sk_orth).
__global__ void __launch_bounds__(NT) k_sk_colnorm(const SkTask* tasks, double* n0, int ldn0) {
  const SkTask t = tasks[blockIdx.y];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int j = blockIdx.x * 4 + wave; j < t.s; j += gridDim.x * 4) {
    const double* y = t.Y + (int64_t)j * t.n;
    double c = 0.0;
    for (int r = lane; r < t.n; r += 64) c += y[r] * y[r];
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0) n0[(int64_t)blockIdx.y * ldn0 + j] = sqrt(c);
  }
}

// Classical Gram-Schmidt with one reorthogonalisation inside a block of 64
// columns of Y (earlier blocks are already projected out).  Column j keeps
// its raw values and a scale sc_j in LDS (q_j = sc_j y_j, sc_j = 0 for a
// dropped column); the scales are applied in one sweep at the end of the
// block.  Per column: dots, update, dots, update fused with the norm, i.e.
// four barriers.  A column whose remaining norm is <= drop times its
// original norm is dropped.
__global__ void __launch_bounds__(NT) k_sk_orth_block(const SkTask* tasks, int j0, double drop, const double* n0, int ldn0) {
  __shared__ double s_c[64], s_sc[64], s_part[NT / 64];
  const SkTask t = tasks[blockIdx.x];
  const int n = t.n, j1 = min(t.s, j0 + 64);
  if (j0 >= t.s) return;
  const auto X = gmem(t.Y);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int j = j0; j < j1; ++j) {
    const auto xj = X + (int64_t)j * n;
    const int cnt = j - j0;
    double part = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      if (cnt > 0) {
        // c_i = q_i^T x_j, four columns per wave at a time
        for (int i0 = 4 * wave; i0 < cnt; i0 += NT / 16) {
          double c[4] = {0.0, 0.0, 0.0, 0.0};
          std::remove_const_t<decltype(X)> xi[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) xi[u] = X + (int64_t)(j0 + min(i0 + u, cnt - 1)) * n;
          // four rows' loads in flight before their products (same order)
          int r = lane;
          for (; r + 192 < n; r += 256) {
            double xv[4], yv[4][4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              xv[q] = xj[r + 64 * q];
#pragma unroll
              for (int u = 0; u < 4; ++u) yv[q][u] = xi[u][r + 64 * q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int u = 0; u < 4; ++u) c[u] += yv[q][u] * xv[q];
          }
          for (; r < n; r += 64) {
            const double v = xj[r];
#pragma unroll
            for (int u = 0; u < 4; ++u) c[u] += xi[u][r] * v;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            double cu = c[u];
            for (int off = 32; off > 0; off >>= 1) cu += __shfl_xor(cu, off, 64);
            if (lane == 0 && i0 + u < cnt) s_c[i0 + u] = cu * s_sc[i0 + u];
          }
        }
        __syncthreads();
      }
      // x_j -= sum_i c_i q_i (and, on the second pass, the squared norm)
      for (int r = tid; r < n; r += NT) {
        double v = xj[r];
        int i = 0;
        for (; i + 8 <= cnt; i += 8) {  // eight loads in flight, then the same sequence of updates
          double xv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) xv[u] = X[r + (int64_t)(j0 + i + u) * n];
#pragma unroll
          for (int u = 0; u < 8; ++u) v -= s_c[i + u] * s_sc[i + u] * xv[u];
        }
        for (; i < cnt; ++i) v -= s_c[i] * s_sc[i] * X[r + (int64_t)(j0 + i) * n];
        if (cnt > 0) xj[r] = v;
        if (pass == 1) part += v * v;
      }
      if (pass == 0 && cnt > 0) __syncthreads();
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if (lane == 0) s_part[wave] = part;
    __syncthreads();
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) tot += s_part[w];
    const double n2 = sqrt(tot);
    const double nn0 = n0[(int64_t)blockIdx.x * ldn0 + j];
    // every thread computes the same value; read by others after the next barrier
    s_sc[cnt] = (n2 > drop * nn0 && n2 > 0.0) ? 1.0 / n2 : 0.0;
  }
  __syncthreads();
  const int nb = j1 - j0;
  if (n > 0) WG_FOR2(n, nb, r, jj) X[r + (int64_t)(j0 + jj) * n] *= s_sc[jj];
  __syncthreads();
}

__global__ void __launch_bounds__(NT) k_sk_trace(const SkTask* tasks) {
  const SkTask t = tasks[blockIdx.x];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < t.n; i += NT) a += t.G[i + (int64_t)i * t.n];
  for (int i = threadIdx.x; i < t.s; i += NT) b += t.B[i + (int64_t)i * t.s];
  const double ta = wg_sum(a);
  const double tb = wg_sum(b);
  if (threadIdx.x == 0) {
    t.tr[0] = ta;
    t.tr[1] = tb;
  }
}

// ok[i] = 1 when sketch i is accepted (see above); cnt from the Ritz values
__global__ void __launch_bounds__(NT) k_sk_check(const SkTask* tasks, const EigTask* et, const int32_t* cnt, double eps2, int32_t* ok,
                           int count) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= count) return;
  const SkTask t = tasks[i];
  const double l0 = et[i].lam[0];
  const double tail = t.tr[0] - t.tr[1];
  // 1 accepted, 0 too narrow (every Ritz value passed), -1 tail too large
  ok[i] = cnt[i] >= t.s ? 0 : ((l0 > 0.0 && tail <= eps2 * l0) ? 1 : -1);
}

// Initial rank reduction, basis step: P2M = V^T, L2P = U, sig = sqrt(lam),
// T = P2Mc V (K x r), S = U^T L2Pc (r x K); then M2M / L2L of the node.
__global__ void __launch_bounds__(NT) k_reduce_basis(LevelView V, int K, const double* work, const int64_t* work_off,
                               const double* m2m8, int has_parent, int sym) {
  const int i = blockIdx.x;
  const int n = V.n[i], r = V.r[i], rc = V.rc[i];
  double* T = V.arena + V.T_off[i];
  double* S = V.arena + V.S_off[i];
  if (n == 0 || r == 0) return;
  const double* base = work + work_off[i];
  // work layout per node: gs, gt (n x n), t (K x n), vs, vt (n x n), ls, lt (n), ws, wt (3n)
  const double* vs = base + 2 * (int64_t)n * n + (int64_t)K * n;
  const double* vt = sym ? vs : vs + (int64_t)n * n;
  const double* ls = vs + 2 * (int64_t)n * n;
  const double* lt = sym ? ls : ls + n;
  double* P2M = V.arena + V.p2m_off[i];
  double* L2P = V.arena + V.l2p_off[i];
  double* sig = V.arena + V.sig_off[i];
  if (r > 0) WG_FOR2(r, n, a, j) {
    P2M[a + (int64_t)j * rc] = vs[j + (int64_t)a * n];
  }
  if (n > 0) WG_FOR2(n, r, j, a) {
    L2P[j + (int64_t)a * n] = vt[j + (int64_t)a * n];
  }
  for (int a = threadIdx.x; a < r; a += NT) {
    sig[a] = sqrt(fmax(ls[a], 0.0));
    sig[rc + a] = sqrt(fmax(lt[a], 0.0));
  }
  __syncthreads();
  wg_gemm(K, r, n, 1.0, V.arena + V.cp2m_off[i], K, false, vs, n, false, 0.0, T, K);
  wg_gemm(r, K, n, 1.0, vt, n, true, V.arena + V.cl2p_off[i], n, false, 0.0, S, rc);
  if (has_parent) {
    const double* M = m2m8 + (int64_t)octant_of(V.coord, i) * K * K;
    wg_gemm(K, r, K, 1.0, M, K, false, T, K, false, 0.0, V.arena + V.m2m_off[i], K);
    wg_gemm(r, K, K, 1.0, S, rc, false, M, K, true, 0.0, V.arena + V.l2l_off[i], rc);
  }
}

// Initial M2L of every interaction pair: M2L_il = (1/L) S_i U_{c_i - c_l} T_l.
__global__ void __launch_bounds__(NT) k_reduce_m2l(LevelView V, int K, const double* unit, double invL, double* tmp, const int64_t* tmp_off) {
  const int i = blockIdx.x;
  const int ri = V.r[i], rci = V.rc[i];
  if (ri == 0) return;
  double* t = tmp + tmp_off[i];
  const double* S = V.arena + V.S_off[i];
  for (int s = V.il_ptr[i]; s < V.il_ptr[i + 1]; ++s) {
    const int l = V.il_idx[s];
    const int rl = V.r[l];
    if (rl == 0) continue;
    const double* U = unit + (int64_t)offset_index(V.coord, i, l) * K * K;
    wg_gemm(K, rl, K, invL, U, K, false, V.arena + V.T_off[l], K, false, 0.0, t, K);
    wg_gemm(ri, rl, K, 1.0, S, rci, false, t, K, false, 0.0, V.il_blk[s], V.ilcap[i]);
  }
}

// The same for K <= 64, one workgroup per (node, group of RM2L_SLOTS
// interaction blocks): U T_l is formed 64 columns at a time in LDS, so no
// global temporary is needed and a few nodes with long lists still fill the chip.
constexpr int RM2L_SLOTS = 4;
__global__ void __launch_bounds__(NT) k_reduce_m2l_lds(LevelView V, int K, const double* unit, double invL) {
  __shared__ double tl[64 * 64];
  const int i = blockIdx.x;
  const int ri = V.r[i], rci = V.rc[i];
  const int s0 = V.il_ptr[i] + blockIdx.y * RM2L_SLOTS, s1 = min(V.il_ptr[i + 1], s0 + RM2L_SLOTS);
  if (ri == 0 || s0 >= s1) return;
  const double* S = V.arena + V.S_off[i];
  for (int s = s0; s < s1; ++s) {
    const int l = V.il_idx[s];
    const int rl = V.r[l];
    const double* U = unit + (int64_t)offset_index(V.coord, i, l) * K * K;
    const double* Tl = V.arena + V.T_off[l];
    for (int c0 = 0; c0 < rl; c0 += 64) {
      const int nc = min(64, rl - c0);
      wg_gemm<false>(K, nc, K, invL, U, K, false, Tl + (int64_t)c0 * K, K, false, 0.0, tl, K);  // C in LDS
      wg_gemm<false>(ri, nc, K, 1.0, S, rci, false, tl, K, false, 0.0, V.il_blk[s] + (int64_t)c0 * V.ilcap[i],
                     V.ilcap[i]);  // B in LDS
    }
  }
}

// ------------------------------------------------------------------ aggregation
// Parent Chebyshev operators: P2Mc_P = [M2M_c ...] (K x n_P), L2Pc_P = [L2L_c; ...].
__global__ void __launch_bounds__(NT) k_agg_cheb(LevelView C, LevelView F, int K, const int32_t* child_ptr, const int32_t* child) {
  const int P = blockIdx.x;
  const int nP = C.n[P];
  double* P2M = C.arena + C.cp2m_off[P];
  double* L2P = C.arena + C.cl2p_off[P];
  int off = 0;
  for (int s = child_ptr[P]; s < child_ptr[P + 1]; ++s) {
    const int c = child[s];
    const int rc = F.r[c], ldc = F.rc[c];
    wg_copy(K, rc, F.arena + F.m2m_off[c], K, P2M + (int64_t)off * K, K);
    wg_copy(rc, K, F.arena + F.l2l_off[c], ldc, L2P + off, nP);
    off += rc;
  }
}

// Parent near block (P, Q) = [M2L_cc'] over the children (near or interaction blocks).
__global__ void __launch_bounds__(NT) k_agg_near(LevelView C, LevelView F, const int32_t* slot_row, const int32_t* child_ptr,
                           const int32_t* child) {
  const int s = blockIdx.x;
  const int P = slot_row[s], Q = C.near_idx[s];
  const int nP = C.n[P];
  double* B = C.arena + C.near_off[s];
  int ro = 0;
  for (int a = child_ptr[P]; a < child_ptr[P + 1]; ++a) {
    const int c = child[a];
    const int rcr = F.r[c];
    int co = 0;
    for (int b = child_ptr[Q]; b < child_ptr[Q + 1]; ++b) {
      const int cc = child[b];
      const int rcc = F.r[cc];
      if (rcr > 0 && rcc > 0) {
        if (dist3(F.coord, c, cc) <= 1) {
          wg_copy(rcr, rcc, F.arena + near_block(F, c, cc), F.n[c], B + ro + (int64_t)co * nP, nP);
        } else {
          wg_copy(rcr, rcc, F.il_blk[il_slot(F, c, cc)], F.ilcap[c], B + ro + (int64_t)co * nP, nP);
        }
      }
      co += rcc;
    }
    ro += rcr;
  }
}

// ------------------------------------------------------------------ phase A
// Pivot D_i = [[P2P_ii, L2P_i], [P2M_i, 0]] and copies of the L- and U-blocks.
// Grid (records, 1 + neighbours, column chunks of GATHER_COLS): part 0 forms
// columns [c0, c0 + GATHER_COLS) of D_i, part 1 + e those of the e-th L- and
// U-blocks, so a few large records still spread over many workgroups.
constexpr int GATHER_COLS = 32;
__device__ inline void wg_copy_cols(int m, int c0, int c1, const double* src, int lds, double* dst, int ldd) {
  if (m > 0 && c1 > c0) wg_copy(m, c1 - c0, src + (int64_t)c0 * lds, lds, dst + (int64_t)c0 * ldd, ldd);
}
__global__ void __launch_bounds__(NT) k_gather(LevelView V, const ElimRec* recs, const ElimNbr* nbrs) {
  const ElimRec R = recs[blockIdx.x];
  const int i = R.node, n = R.n, r = R.r, d = R.d;
  const int c0 = blockIdx.z * GATHER_COLS, c1 = c0 + GATHER_COLS;
  const int part = blockIdx.y;
  if (part == 0) {
    if (c0 >= d) return;
    const int rc = V.rc[i];
    // columns [0, n): P2P_ii over P2M_i; columns [n, d): L2P_i over zeros
    const int a = c0, b = min(c1, n);
    wg_copy_cols(n, a, b, V.arena + near_block(V, i, i), n, R.lu, d);
    wg_copy_cols(r, a, b, V.arena + V.p2m_off[i], rc, R.lu + n, d);
    const int a2 = max(c0, n) - n, b2 = min(c1, d) - n;
    wg_copy_cols(n, a2, b2, V.arena + V.l2p_off[i], n, R.lu + (int64_t)n * d, d);
    if (r > 0 && b2 > a2) wg_fill(r, b2 - a2, R.lu + n + (int64_t)(n + a2) * d, d, 0.0);
    return;
  }
  if (part > R.nnb) return;
  const ElimNbr B = nbrs[R.nb_begin + part - 1];
  const int np = V.n[B.p];
  wg_copy_cols(B.m, c0, min(c1, n), V.arena + B.blk_pi, np, R.L + B.off, R.M);
  wg_copy_cols(n, c0, min(c1, B.m), V.arena + B.blk_ip, n, R.U + (int64_t)B.off * n, n);
}

__global__ void __launch_bounds__(NT) k_getrf(const ElimRec* recs, int32_t* info, int big_d) {
  const ElimRec R = recs[blockIdx.x];
  if (R.d >= big_d) return;  // blocked path
  const int inf = wg_getrf(R.d, R.lu, R.d, R.piv);
  if (threadIdx.x == 0) info[blockIdx.x] = inf;
}

// X = D^-1 [[U, 0, I_n], [0, I_r, 0]]  (d x (M + r + n)), XCOLS columns per
// workgroup: the Schur update takes the first M + r columns, the solve the
// explicit inverse (the last r + n columns) and the x-rows of the first M.
// Pivots of order <= DMAX keep their slice of X in LDS through the row
// interchanges and both substitutions (2 d barrier steps, all on LDS); larger
// ones solve in place in global memory.  DMAX sizes the LDS (occupancy).
constexpr int XCOLS = 32;
struct XTask {
  int32_t rec, c0;
};
template <int DMAX>
__global__ void __launch_bounds__(NT) k_xsolve(const ElimRec* recs, const XTask* xt) {
  __shared__ double xs[DMAX * XCOLS];
  const XTask t = xt[blockIdx.x];
  const ElimRec R = recs[t.rec];
  const int n = R.n, d = R.d, M = R.M;
  const int nc = min(XCOLS, M + R.r + n - t.c0);
  if (d == 0 || nc <= 0) return;
  double* X = R.X + (int64_t)t.c0 * d;
  const bool lds = d <= DMAX;
  double* B = lds ? xs : X;  // ld d either way
  WG_FOR2(d, nc, row, cl) {
    const int col = t.c0 + cl;
    double v;
    if (col < M) v = row < n ? R.U[row + (int64_t)col * n] : 0.0;
    else if (col < M + R.r) v = (row >= n && row - n == col - M) ? 1.0 : 0.0;
    else v = (row == col - M - R.r) ? 1.0 : 0.0;
    B[row + cl * d] = v;
  }
  __syncthreads();
  wg_getrs(d, R.lu, d, R.piv, B, d, nc);
  if (lds) {
    WG_FOR2(d, nc, row, cl) X[row + (int64_t)cl * d] = xs[row + cl * d];
    __syncthreads();
  }
}

// The same solve for pivots of order d <= NT with one row per thread: thread i
// keeps row i of its 32-column slice in registers through both substitutions.
// The row interchanges become one permutation first (row i of P B is row
// perm[i] of B); per pivot row j the row goes through LDS to the others, and
// each thread's multiplier of the next step is loaded during the current one.
// Every element sees the same operations in the same order as in wg_getrs.
__global__ void __launch_bounds__(NT) k_xsolve_rows(const ElimRec* recs, const XTask* xt) {
  __shared__ double rowj[XCOLS];
  __shared__ int32_t perm[NT], spiv[NT];
  const XTask t = xt[blockIdx.x];
  const ElimRec R = recs[t.rec];
  const int n = R.n, d = R.d, M = R.M, r = R.r;
  const int nc = min(XCOLS, M + r + n - t.c0);
  if (d == 0 || nc <= 0) return;
  const int i = threadIdx.x;
  const bool own = i < d;
  const auto LU = gmem(R.lu);
  if (own) {
    perm[i] = i;
    spiv[i] = R.piv[i];
  }
  __syncthreads();
  if (i == 0)
    for (int j = 0; j < d; ++j) {
      const int p = spiv[j];
      if (p != j) {
        const int a = perm[j];
        perm[j] = perm[p];
        perm[p] = a;
      }
    }
  __syncthreads();
  // row perm[i] of X0 = [[U, 0, I_n], [0, I_r, 0]] in columns c0 .. c0+nc-1
  const int row = own ? perm[i] : 0;
  double x[XCOLS];
#pragma unroll
  for (int c = 0; c < XCOLS; ++c) {
    const int col = t.c0 + c;
    double v = 0.0;
    if (own && c < nc) {
      if (col < M) v = row < n ? R.U[row + (int64_t)col * n] : 0.0;
      else if (col < M + r) v = (row >= n && row - n == col - M) ? 1.0 : 0.0;
      else v = (row == col - M - r) ? 1.0 : 0.0;
    }
    x[c] = v;
  }
  // forward: unit lower, x_i -= L[i][j] x_j for i > j
  double l_next = (own && i > 0) ? LU[i] : 0.0;
  for (int j = 0; j + 1 < d; ++j) {
    const double l = l_next;
    if (i == j)
#pragma unroll
      for (int c = 0; c < XCOLS; ++c) rowj[c] = x[c];
    __syncthreads();
    l_next = (own && i > j + 1) ? LU[i + (int64_t)(j + 1) * d] : 0.0;
    if (own && i > j)
#pragma unroll
      for (int c = 0; c < XCOLS; ++c) x[c] -= l * rowj[c];
    __syncthreads();
  }
  // backward: upper, x_j /= U[j][j], then x_i -= U[i][j] x_j for i < j
  double u_next = (own && i < d - 1) ? LU[i + (int64_t)(d - 1) * d] : 0.0;
  const double dii = own ? LU[i + (int64_t)i * d] : 1.0;  // this row's pivot, loaded ahead
  for (int j = d - 1; j >= 0; --j) {
    const double u = u_next;
    if (i == j) {
#pragma unroll
      for (int c = 0; c < XCOLS; ++c) x[c] /= dii;
#pragma unroll
      for (int c = 0; c < XCOLS; ++c) rowj[c] = x[c];
    }
    __syncthreads();
    u_next = (own && j > 0 && i < j - 1) ? LU[i + (int64_t)(j - 1) * d] : 0.0;
    if (own && i < j)
#pragma unroll
      for (int c = 0; c < XCOLS; ++c) x[c] -= u * rowj[c];
    __syncthreads();
  }
  if (own) {
    const auto X = gmem(R.X + (int64_t)t.c0 * d);
#pragma unroll
    for (int c = 0; c < XCOLS; ++c)
      if (c < nc) X[i + (int64_t)c * d] = x[c];
  }
}

// ---- large pivots: right-looking blocked LU of the augmented matrix
// [D | X0] (d x (d + W)), X0 = [[U, 0], [0, I]], pivoting over the columns of
// D only.  The trailing updates carry L^-1 P X0 along in the X columns; a
// blocked backward substitution with U then leaves X = D^-1 X0.  Every step
// is one launch over all large pivots of a colour, many workgroups each, so
// a colour with a handful of big nodes still fills the device.  Panel width
// 64; the panel itself is factorised by one workgroup.  piv follows the
// convention of wg_getrf, so the solve phase reads the factors unchanged.
constexpr int BLU_NB = 64;
constexpr int BD_MAXN = 4096;  // largest box of the block-diagonal preconditioner
constexpr int BLU_NB_PAD = BLU_NB + 1;

struct BluTask {
  double* lu;
  double* X;
  int32_t* piv;
  int32_t* info;
  double* dinv;  // inverses of the 64 x 64 diagonal blocks: L11^-1 (unit lower) / U11^-1 per panel, 64 x 64 each
  int32_t d, W;
};

// Inverse of a triangular nb x nb diagonal block T (in LDS) into Inv (global,
// ld 64): lower = 1: unit lower triangular; lower = 0: upper triangular with
// its diagonal.  Column c of the inverse solves T x = e_c by substitution, one
// thread per column, the columns held in LDS.
__device__ inline void wg_tri_inverse(const double (*T)[BLU_NB_PAD], int nb, int lower, double* Inv) {
  __shared__ double Xs[BLU_NB][BLU_NB_PAD];
  const int c = threadIdx.x;
  if (c < nb) {
    if (lower) {
      for (int i = 0; i < nb; ++i) {
        double v = (i == c) ? 1.0 : 0.0;
        for (int q = c; q < i; ++q) v -= T[i][q] * Xs[q][c];
        Xs[i][c] = i < c ? 0.0 : v;
      }
    } else {
      for (int i = nb - 1; i >= 0; --i) {
        double v = (i == c) ? 1.0 : 0.0;
        if (i <= c) {
          for (int q = i + 1; q <= c; ++q) v -= T[i][q] * Xs[q][c];
          v /= T[i][i];
        } else {
          v = 0.0;
        }
        Xs[i][c] = v;
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = e & 63, j = e >> 6;
    Inv[i + 64 * j] = (i < nb && j < nb) ? Xs[i][j] : 0.0;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(NT) k_blu_xinit(const BluTask* tasks, const ElimRec* recs, const int32_t* rec_of) {
  const BluTask t = tasks[blockIdx.y];
  const ElimRec R = recs[rec_of[blockIdx.y]];
  const int c0 = blockIdx.x * 64;
  const int nc = min(64, t.W - c0);
  if (threadIdx.x == 0 && blockIdx.x == 0) *t.info = 0;
  if (nc <= 0 || t.d == 0) return;
  const int n = R.n, M = R.M, r = R.r;
  WG_FOR2(t.d, nc, row, cl) {
    const int col = c0 + cl;
    double v;
    if (col < M) v = row < n ? R.U[row + (int64_t)col * n] : 0.0;
    else if (col < M + r) v = (row >= n && row - n == col - M) ? 1.0 : 0.0;
    else v = (row == col - M - r) ? 1.0 : 0.0;  // [I_n; 0]: the x-columns of D^-1
    t.X[row + (int64_t)col * t.d] = v;
  }
}

// Panel LU of columns j0 .. j0+nb-1 over rows j0 .. d-1, one workgroup per
// task.  Per column: the pivot (largest magnitude, first on ties), the row
// interchange inside the panel, the scaling of the column and the rank-1
// update of the panel columns to its right.  The scaling and the update go
// through their elements four per thread at a time, loads first, then the
// arithmetic, then the stores, so that a batch of loads is in flight at once
// (a wait for a load issued after a store also waits for the store).
__global__ void __launch_bounds__(NT) k_blu_panel(const BluTask* tasks, int j0) {
  const BluTask t = tasks[blockIdx.x];
  const int d = t.d;
  if (j0 >= d) return;
  const int nb = min(BLU_NB, d - j0);
  double* T = t.lu;
  const auto Tg = gmem(T);
  const int tid = threadIdx.x;
  for (int j = j0; j < j0 + nb; ++j) {
    double best = -1.0;
    int bi = j;  // in range even for a NaN column
    for (int i = j + tid; i < d; i += NT) {
      const double v = fabs(Tg[i + (int64_t)j * d]);
      if (v > best) { best = v; bi = i; }
    }
    wg_argmax(best, bi);
    const int p = bi;
    const double pv = best;
    if (tid == 0) {
      t.piv[j] = p;
      if (pv == 0.0 && *t.info == 0) *t.info = j + 1;
    }
    if (p != j)
      for (int c = j0 + tid; c < j0 + nb; c += NT) {
        const double x = T[j + (int64_t)c * d];
        T[j + (int64_t)c * d] = T[p + (int64_t)c * d];
        T[p + (int64_t)c * d] = x;
      }
    __syncthreads();
    const double dj = T[j + (int64_t)j * d];
    if (dj != 0.0)
      for (int i0 = j + 1; i0 < d; i0 += 4 * NT) {
        double x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0 + tid + NT * q;
          x[q] = i < d ? Tg[i + (int64_t)j * d] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] /= dj;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0 + tid + NT * q;
          if (i < d) Tg[i + (int64_t)j * d] = x[q];
        }
      }
    __syncthreads();
    const int rem = d - j - 1, w = j0 + nb - j - 1;
    if (rem > 0 && w > 0) {
      // element e = ii + rem * cc of the rem x w block, e = tid + NT * step;
      // (ii, cc) advance by NT per step without a division
      const int di = NT % rem, dc = NT / rem;
      int ii = tid % rem, cc = tid / rem;
      while (cc < w) {
        int ri[4], ci[4];
        double x[4], l[4], u[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          ri[q] = ii;
          ci[q] = cc;
          ii += di;
          cc += dc;
          if (ii >= rem) { ii -= rem; ++cc; }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const bool ok = ci[q] < w;
          const int64_t col = (int64_t)(j + 1 + (ok ? ci[q] : 0)) * d;
          x[q] = ok ? Tg[j + 1 + ri[q] + col] : 0.0;
          l[q] = ok ? Tg[j + 1 + ri[q] + (int64_t)j * d] : 0.0;
          u[q] = ok ? Tg[j + col] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] -= l[q] * u[q];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (ci[q] < w) Tg[j + 1 + ri[q] + (int64_t)(j + 1 + ci[q]) * d] = x[q];
      }
    }
    __syncthreads();
  }
  // L11^-1 of this panel for the block triangular solve of the columns to its right
  __shared__ double Ls[BLU_NB][BLU_NB_PAD];
  for (int e = tid; e < nb * nb; e += NT) Ls[e % nb][e / nb] = T[j0 + e % nb + (int64_t)(j0 + e / nb) * d];
  __syncthreads();
  wg_tri_inverse(Ls, nb, 1, t.dinv + (int64_t)(j0 / BLU_NB) * 2 * 4096);
}

// U_jj^-1 of every diagonal block (after the factorisation), grid (blocks, tasks)
__global__ void __launch_bounds__(NT) k_blu_uinv(const BluTask* tasks) {
  __shared__ double Us[BLU_NB][BLU_NB_PAD];
  const BluTask t = tasks[blockIdx.y];
  const int j0 = blockIdx.x * BLU_NB;
  if (j0 >= t.d) return;
  const int nb = min(BLU_NB, t.d - j0);
  for (int e = threadIdx.x; e < nb * nb; e += NT) Us[e % nb][e / nb] = t.lu[j0 + e % nb + (int64_t)(j0 + e / nb) * t.d];
  __syncthreads();
  wg_tri_inverse(Us, nb, 0, t.dinv + (int64_t)blockIdx.x * 2 * 4096 + 4096);
}

// columns outside the panel: c < d in lu, c >= d in X (both leading dim d)
__device__ inline double* blu_col(const BluTask& t, int c) {
  return c < t.d ? t.lu + (int64_t)c * t.d : t.X + (int64_t)(c - t.d) * t.d;
}

__global__ void __launch_bounds__(NT) k_blu_swap(const BluTask* tasks, int j0) {
  const BluTask t = tasks[blockIdx.y];
  const int d = t.d;
  if (j0 >= d) return;
  const int nb = min(BLU_NB, d - j0);
  const int c = blockIdx.x * NT + threadIdx.x;
  if (c >= d + t.W || (c >= j0 && c < j0 + nb)) return;
  double* col = blu_col(t, c);
  for (int j = j0; j < j0 + nb; ++j) {
    const int p = t.piv[j];
    if (p != j) {
      const double x = col[j];
      col[j] = col[p];
      col[p] = x;
    }
  }
}

// column chunks right of the panel: first the lu columns j0+nb..d-1, then the
// X columns, each split into chunks of 64 that never straddle the two
__device__ inline int blu_chunks_lu(const BluTask& t, int j0, int nb) { return (t.d - j0 - nb + 63) / 64; }

__global__ void __launch_bounds__(NT) k_blu_trsm(const BluTask* tasks, int j0) {
  const BluTask t = tasks[blockIdx.y];
  const int d = t.d;
  if (j0 >= d) return;
  const int nb = min(BLU_NB, d - j0);
  const int clu = blu_chunks_lu(t, j0, nb);
  const int cx = (t.W + 63) / 64;
  const int ch = blockIdx.x;
  if (ch >= clu + cx) return;
  int c0, nc;
  double* base;
  if (ch < clu) {
    c0 = j0 + nb + ch * 64; nc = min(64, d - c0); base = t.lu;
  } else {
    c0 = (ch - clu) * 64; nc = min(64, t.W - c0); base = t.X;
  }
  // U12 = L11^-1 A12 in place: one 64 x 64 output tile whose operand is read
  // completely before the tile is written
  wg_gemm(nb, nc, nb, 1.0, t.dinv + (int64_t)(j0 / BLU_NB) * 2 * 4096, 64, false, base + j0 + (int64_t)c0 * d, d,
          false, 0.0, base + j0 + (int64_t)c0 * d, d);
}

// trailing update A22 -= L21 U12 over the lu columns right of the panel and
// all X columns; grid (row tiles, column chunks, task)
__global__ void __launch_bounds__(NT) k_blu_gemm(const BluTask* tasks, int j0) {
  const BluTask t = tasks[blockIdx.z];
  const int d = t.d;
  if (j0 >= d) return;
  const int nb = min(BLU_NB, d - j0);
  const int r0 = j0 + nb + blockIdx.x * 64;
  if (r0 >= d) return;
  const int clu = blu_chunks_lu(t, j0, nb);
  const int cx = (t.W + 63) / 64;
  const int ch = blockIdx.y;
  if (ch >= clu + cx) return;
  int c0, nc;
  double* base;
  if (ch < clu) {
    c0 = j0 + nb + ch * 64; nc = min(64, d - c0); base = t.lu;
  } else {
    c0 = (ch - clu) * 64; nc = min(64, t.W - c0); base = t.X;
  }
  const int mr = min(64, d - r0);
  wg_gemm(mr, nc, nb, -1.0, t.lu + r0 + (int64_t)j0 * d, d, false, base + j0 + (int64_t)c0 * d, d, false, 1.0,
          base + r0 + (int64_t)c0 * d, d);
}

// backward substitution, block row jb: X_jb = U_jb,jb^-1 X_jb (per 64 columns, in place)
__global__ void __launch_bounds__(NT) k_bu_trsm(const BluTask* tasks, int jb) {
  const BluTask t = tasks[blockIdx.y];
  const int d = t.d, j0 = jb * BLU_NB;
  if (j0 >= d) return;
  const int nb = min(BLU_NB, d - j0);
  const int c0 = blockIdx.x * 64;
  if (c0 >= t.W) return;
  const int nc = min(64, t.W - c0);
  wg_gemm(nb, nc, nb, 1.0, t.dinv + (int64_t)jb * 2 * 4096 + 4096, 64, false, t.X + j0 + (int64_t)c0 * d, d, false,
          0.0, t.X + j0 + (int64_t)c0 * d, d);
}

// X[0:j0, :] -= U[0:j0, j0:j0+nb] X[j0:j0+nb, :]; grid (row tiles, column chunks, task)
__global__ void __launch_bounds__(NT) k_bu_gemm(const BluTask* tasks, int jb) {
  const BluTask t = tasks[blockIdx.z];
  const int d = t.d, j0 = jb * BLU_NB;
  if (j0 >= d) return;
  const int nb = min(BLU_NB, d - j0);
  const int r0 = blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  if (r0 >= j0 || c0 >= t.W) return;
  const int mr = min(64, j0 - r0), nc = min(64, t.W - c0);
  wg_gemm(mr, nc, nb, -1.0, t.lu + r0 + (int64_t)j0 * d, d, false, t.X + j0 + (int64_t)c0 * d, d, false, 1.0,
          t.X + r0 + (int64_t)c0 * d, d);
}

// Schur-complement update of one row block a of the neighbours of i (a == nnb:
// the surviving row R_z_i of i itself), for one column block b (b == -1: the
// new column C_y_i; b == -2: every column block, the small-node form).
//   near (dist <= 1):  M[p, q] -= L_a X_top[:, q]
//   far  (dist 2):     F_ab = -L_a X_top[:, q]          (compressed later)
//   new blocks:        M[p, i] = L_a F,  M[i, q] = X_bot[:, q],  M[i, i] = -H
// (with n == 0 the products are empty: far blocks become zero, near blocks
// stay, the new block is zero)
// tile: -1 = the whole block; else ti | tj << 16, the 64 x 64 output tile
// (rows 64 ti, columns 64 tj) of block (a, b), a < nnb, b >= -1
struct SchurTask {
  int32_t rec, a, b, tile;
};
// product of the Schur update: FP64, FP32 lite tile, or FP32 with the
// double-buffered tile for long inner dimensions (own kernel instances).
// In the mixed form only the far fill-in F = -L_a X_b goes through FP32: it
// is formed fresh (no cancellation against stored data) and then compressed
// at relative accuracy eps.  The near blocks are updated in place, M -= L X,
// where the difference can be far smaller than either term, and stay FP64.
// FP64 products go to the FP64 matrix-core tile in the instances with mf set,
// to the FMA tile without (both take the one-pass product below 32 x 32 x 32).
// A template parameter, not a runtime switch, so that one tile's registers do
// not lower the other instances' occupancy.
template <bool f32, bool deep, bool mf>
__device__ inline void schur_gemm(int m, int n, int k, double alpha, const double* A, int lda, const double* B,
                                  int ldb, double beta, double* C, int ldc) {
  if (!f32 && mf) wg_gemm_f64m(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
  else if (!f32) wg_gemm(m, n, k, alpha, A, lda, false, B, ldb, false, beta, C, ldc);
  else if (deep) wg_gemm_f32_deep(m, n, k, alpha, A, lda, false, B, ldb, false, beta, C, ldc);
  else wg_gemm_f32(m, n, k, alpha, A, lda, false, B, ldb, false, beta, C, ldc);
}
// One product of the Schur update, C = alpha A B + beta C: far (a fill-in
// block, formed fresh) or near (a stored block updated in place).
struct SchurProd {
  int m, n, k, lda, ldb, ldc;
  double alpha, beta;
  const double* A;
  const double* B;
  double* C;
  bool far;
};
// The product of block (a, b) of the update of record R, a < nnb; b = -1 is
// the new block (p, i) = L_a F with [F; H] = D^-1 [0; I].  With tj >= 0 only
// the 64 x 64 output tile (ti, tj) of it.
__device__ inline SchurProd schur_prod(const LevelView& V, const ElimRec& R, const ElimNbr* nbrs,
                                       const int32_t* far_idx, const FarPair* far, int a, int b, int ti, int tj) {
  const int n = R.n, d = R.d, M = R.M;
  const ElimNbr A = nbrs[R.nb_begin + a];
  const int np = V.n[A.p];
  const int i0 = tj >= 0 ? 64 * ti : 0, j0 = tj >= 0 ? 64 * tj : 0;
  SchurProd P;
  P.m = tj >= 0 ? min(64, A.m - i0) : A.m;
  P.k = n;
  P.A = R.L + A.off + i0;
  P.lda = M;
  P.ldb = d;
  if (b >= 0) {
    const ElimNbr B = nbrs[R.nb_begin + b];
    P.n = tj >= 0 ? min(64, B.m - j0) : B.m;
    P.B = R.X + (int64_t)(B.off + j0) * d;
    P.alpha = -1.0;
    const int fi = far_idx[R.far_base + a * R.nnb + b];
    P.far = fi >= 0;
    if (fi < 0) {
      P.C = V.arena + near_block(V, A.p, B.p) + i0 + (int64_t)j0 * np;
      P.ldc = np;
      P.beta = 1.0;
    } else {
      P.C = far[fi].F + i0 + (int64_t)j0 * A.m;
      P.ldc = A.m;
      P.beta = 0.0;
    }
  } else {
    P.n = tj >= 0 ? min(64, R.r - j0) : R.r;
    P.B = R.X + (int64_t)(M + j0) * d;
    P.alpha = 1.0;
    P.beta = 0.0;
    P.C = V.arena + A.blk_pi + i0 + (int64_t)j0 * np;
    P.ldc = np;
    P.far = false;
  }
  return P;
}
// The row R_z_i of the update (a = nnb): copies of X's rows, no products.
__device__ inline void schur_copy(const LevelView& V, const ElimRec& R, const ElimNbr* nbrs, int b) {
  const int n = R.n, r = R.r, d = R.d, M = R.M;
  if (b >= 0) {
    const ElimNbr B = nbrs[R.nb_begin + b];
    wg_copy(r, B.m, R.X + n + (int64_t)B.off * d, d, V.arena + B.blk_ip, n);
  } else {
    wg_copy(r, r, R.X + n + (int64_t)M * d, d, V.arena + near_block(V, R.node, R.node), n, -1.0);
  }
}

// One task per workgroup: a 64 x 64 output tile of block (a, b), a block
// (a, b), or a whole row block a (b = -2, its blocks one after the other).
// Every product goes through one of two call sites (far in the mixed form:
// FP32 tile; otherwise FP64), so each tile is inlined once.  part: 0 every
// product, 1 the near products and the copies only, 2 the far products only
// (the mixed form runs 1 and 2 as two kernels, each with one tile's
// registers, at the same time on two streams).
template <bool f32, bool deep, bool mf, int part>
__global__ void __launch_bounds__(NT) k_schur(LevelView V, const ElimRec* recs, const ElimNbr* nbrs,
                                              const SchurTask* tasks, const int32_t* far_idx, const FarPair* far) {
  const SchurTask T = tasks[blockIdx.x];
  const ElimRec R = recs[T.rec];
  const int tile = T.tile;
  // a row block: its blocks 0..nnb-1, then the new block (b = -1)
  const int nb = T.b == -2 ? R.nnb + 1 : 1;
  for (int q = 0; q < nb; ++q) {
    const int b = T.b == -2 ? (q < R.nnb ? q : -1) : T.b;
    if (T.a >= R.nnb) {
      if (part != 2) schur_copy(V, R, nbrs, b);
      continue;
    }
    const SchurProd P = schur_prod(V, R, nbrs, far_idx, far, T.a, b, tile >= 0 ? (tile & 0xffff) : 0,
                                   tile >= 0 ? (tile >> 16) : -1);
    if ((part == 1 && P.far) || (part == 2 && !P.far)) continue;
    if (part == 2 || (part == 0 && f32 && P.far))
      schur_gemm<true, deep, false>(P.m, P.n, P.k, P.alpha, P.A, P.lda, P.B, P.ldb, P.beta, P.C, P.ldc);
    else
      schur_gemm<false, false, mf>(P.m, P.n, P.k, P.alpha, P.A, P.lda, P.B, P.ldb, P.beta, P.C, P.ldc);
  }
}

// Gram matrices of a changed node p (side 0: source, side 1: target):
//   Gs = P2M^T diag(sig_s^2) P2M + sum_q F_qp^T F_qp
//   Gt = L2P diag(sig_t^2) L2P^T + sum_q F_pq F_pq^T
// Scaled bases of a changed node, one workgroup per (node, side):
//   side 0: t0 = diag(sig_s) P2M (r x n);  side 1: t1 = L2P diag(sig_t) (n x r)
// (the two sides use disjoint halves of the node's tmp buffer)
__global__ void __launch_bounds__(NT) k_gram_prep(LevelView V, const Changed* chg, int sides) {
  const Changed C = chg[sides == 2 ? blockIdx.x >> 1 : blockIdx.x];
  const int side = sides == 2 ? (int)(blockIdx.x & 1) : 0;
  const int p = C.p, n = C.n, r = C.r, rc = V.rc[p];
  const double* sig = V.arena + V.sig_off[p];
  double* t = C.tmp + (int64_t)side * r * n;
  if (r == 0 || n == 0) return;
  if (side == 0) {
    const double* P2M = V.arena + V.p2m_off[p];
    wg_each2(r, n, [&](int a, int j) { return make_double2(sig[a], P2M[a + (int64_t)j * rc]); },
             [&](int a, int j, double2 v) { t[a + (int64_t)j * r] = v.x * v.y; });
  } else {
    const double* L2P = V.arena + V.l2p_off[p];
    wg_each2(n, r, [&](int j, int a) { return make_double2(L2P[j + (int64_t)a * n], sig[rc + a]); },
             [&](int j, int a, double2 v) { t[j + (int64_t)a * n] = v.x * v.y; });
  }
}

// Gram matrices of a changed node p (side 0: source, side 1: target):
//   Gs = t0^T t0 + sum_q F_qp^T F_qp,   Gt = t1 t1^T + sum_q F_pq F_pq^T
// One workgroup per 64 x 64 tile of the lower triangle (grid.x), mirrored
// into the upper one; grid.y = (node, side).
__global__ void __launch_bounds__(NT) k_gram(LevelView V, const Changed* chg, const FarRef* refs, const FarPair* far,
                       const ElimNbr* nbrs, const ElimRec* recs, int sides) {
  const Changed C = chg[sides == 2 ? blockIdx.y >> 1 : blockIdx.y];
  const int side = sides == 2 ? (int)(blockIdx.y & 1) : 0;
  const int n = C.n, r = C.r;
  const int nb = (n + 63) / 64;
  const int tile = blockIdx.x;
  if (tile >= nb * (nb + 1) / 2) return;
  int ti = (int)((sqrt(8.0 * tile + 1.0) - 1.0) * 0.5);
  while (ti * (ti + 1) / 2 > tile) --ti;
  while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
  const int tj = tile - ti * (ti + 1) / 2;
  const int I = ti * 64, J = tj * 64;
  const int mi = min(64, n - I), mj = min(64, n - J);
  double* G = side ? C.gt : C.gs;
  const double* t = C.tmp + (int64_t)side * r * n;
  const ElimRec R = recs[C.rec];
  if (side == 0) {
    wg_gemm(mi, mj, r, 1.0, t + (int64_t)I * r, r, true, t + (int64_t)J * r, r, false, 0.0, G + I + (int64_t)J * n, n);
    for (int k = 0; k < C.far_count; ++k) {
      const FarPair Pq = far[refs[C.far_begin + k].ba];  // rows of q, columns of p
      const int mq = nbrs[R.nb_begin + Pq.a].m;
      wg_gemm(mi, mj, mq, 1.0, Pq.F + (int64_t)I * mq, mq, true, Pq.F + (int64_t)J * mq, mq, false, 1.0,
              G + I + (int64_t)J * n, n);
    }
  } else {
    wg_gemm(mi, mj, r, 1.0, t + I, n, false, t + J, n, true, 0.0, G + I + (int64_t)J * n, n);
    for (int k = 0; k < C.far_count; ++k) {
      const FarPair Pq = far[refs[C.far_begin + k].ab];  // rows of p, columns of q
      const int mq = nbrs[R.nb_begin + Pq.b].m;
      wg_gemm(mi, mj, mq, 1.0, Pq.F + I, n, false, Pq.F + J, n, true, 1.0, G + I + (int64_t)J * n, n);
    }
  }
  if (ti != tj) {
    const auto Gg = gmem(G);
    wg_each2(mi, mj, [&](int a, int b) { return Gg[I + a + (int64_t)(J + b) * n]; },
             [&](int a, int b, double v) { Gg[J + b + (int64_t)(I + a) * n] = v; });
  }
}

// New bases of a changed node: V' = leading rnew eigenvectors of Gs, U' of Gt;
// T_p = P2M V' (r x rnew), S_p = U'^T L2P (rnew x r); then overwrite the bases.
__global__ void __launch_bounds__(NT) k_basis(LevelView V, const Changed* chg) {
  const Changed C = chg[blockIdx.x];
  const int p = C.p, n = C.n, r = C.r, rn = C.rnew, rc = V.rc[p];
  double* P2M = V.arena + V.p2m_off[p];
  double* L2P = V.arena + V.l2p_off[p];
  double* sig = V.arena + V.sig_off[p];
  wg_gemm(r, rn, n, 1.0, P2M, rc, false, C.vs, n, false, 0.0, C.T, r > 0 ? r : 1);
  wg_gemm(rn, r, n, 1.0, C.vt, n, true, L2P, n, false, 0.0, C.S, rn > 0 ? rn : 1);
  wg_each2(rn, n, [&](int a, int j) { return C.vs[j + (int64_t)a * n]; },
           [&](int a, int j, double v) { P2M[a + (int64_t)j * rc] = v; });
  wg_each2(n, rn, [&](int j, int a) { return C.vt[j + (int64_t)a * n]; },
           [&](int j, int a, double v) { L2P[j + (int64_t)a * n] = v; });
  for (int a = threadIdx.x; a < rn; a += NT) {
    sig[a] = sqrt(fmax(C.ls[a], 0.0));
    sig[rc + a] = sqrt(fmax(C.lt[a], 0.0));
  }
  __syncthreads();
}

// Projection of a far fill-in onto the new bases (the final block is left in
// F with leading dimension = its row count):
//   both changed   F <- U_a'^T F V_b'     a changed   F <- U_a'^T F
//   b changed      F <- F V_b'            both eliminated: M2L_ab += F
// U_a' = L2P_a (n_a x r_a', ld n_a), V_b' = P2M_b^T (P2M_b: r_b' x n_b, ld rc_b).
__global__ void __launch_bounds__(NT) k_project(LevelView V, const FarPair* far, const ElimRec* recs, const ElimNbr* nbrs,
                          const Changed* chg) {
  const FarPair P = far[blockIdx.x];
  const ElimRec R = recs[P.rec];
  const ElimNbr A = nbrs[R.nb_begin + P.a], B = nbrs[R.nb_begin + P.b];
  if (P.direct) {
    double* dst = P.dst;
    wg_add(A.m, B.m, P.F, A.m, dst, P.dst_ld);
    return;
  }
  const int ra = A.elim ? A.m : chg[V.chg[A.p]].rnew;
  const int rb = B.elim ? B.m : chg[V.chg[B.p]].rnew;
  if (!A.elim && !B.elim) {
    wg_gemm(ra, B.m, A.m, 1.0, V.arena + V.l2p_off[A.p], A.m, true, P.F, A.m, false, 0.0, P.D, ra > 0 ? ra : 1);
    wg_gemm(ra, rb, B.m, 1.0, P.D, ra > 0 ? ra : 1, false, V.arena + V.p2m_off[B.p], V.rc[B.p], true, 0.0, P.F,
            ra > 0 ? ra : 1);
  } else if (!A.elim) {
    wg_gemm(ra, B.m, A.m, 1.0, V.arena + V.l2p_off[A.p], A.m, true, P.F, A.m, false, 0.0, P.D, ra > 0 ? ra : 1);
    wg_copy(ra, B.m, P.D, ra > 0 ? ra : 1, P.F, ra > 0 ? ra : 1);
  } else {
    wg_gemm(A.m, rb, B.m, 1.0, P.F, A.m, false, V.arena + V.p2m_off[B.p], V.rc[B.p], true, 0.0, P.D, A.m);
    wg_copy(A.m, rb, P.D, A.m, P.F, A.m);
  }
}

__device__ inline int find_ref(const FarRef* refs, int begin, int count, int q) {
  for (int k = 0; k < count; ++k)
    if (refs[begin + k].q == q) return begin + k;
  return -1;
}

// Phase B: push the basis change of a changed node p into the M2L blocks of its
// interaction list, into M2M_p and L2L_p, and add the projected fill-ins.
// Owner rule: block (t, s) is transformed by t's workgroup when t changed,
// else by s's, so every block is written once.
//   (p, l):              S_p M (T_l if l changed) + D_pl
//   (l, p), l unchanged: M T_p + D_lp
// A block whose capacity grew is read from its old storage (blk_old, ld
// cap_old) and written to its new one (V.il_blk, ld V.ilcap).
// k_phase_b: one workgroup per changed node (small ranks).
template <bool f32>
__global__ void __launch_bounds__(NT) k_phase_b(LevelView V, int K, const Changed* chg, const FarRef* refs,
                                                const FarPair* far, int has_parent, double* const* blk_old,
                                                const int32_t* cap_old) {
  const Changed C = chg[blockIdx.x];
  const int p = C.p, r = C.r, rn = C.rnew, rcp = V.rc[p];
  double* t = C.tmp;
  for (int s = V.il_ptr[p]; s < V.il_ptr[p + 1]; ++s) {
    const int l = V.il_idx[s];
    const int rl = V.r[l];
    const int lc = V.chg[l];
    const double* Mo = blk_old[s];
    double* M = V.il_blk[s];
    const int ldo = cap_old[p], ldn = V.ilcap[p];
    const int rln = lc >= 0 ? chg[lc].rnew : rl;
    // t = M (T_l)   (r x rln, ld r)
    if (lc >= 0) wg_gemm_p(f32, r, rln, rl, 1.0, Mo, ldo, false, chg[lc].T, rl > 0 ? rl : 1, false, 0.0, t, r > 0 ? r : 1);
    else wg_copy(r, rl, Mo, ldo, t, r > 0 ? r : 1);
    // M = S_p t   (rn x rln)
    wg_gemm_p(f32, rn, rln, r, 1.0, C.S, rn > 0 ? rn : 1, false, t, r > 0 ? r : 1, false, 0.0, M, ldn);
    const int k = find_ref(refs, C.far_begin, C.far_count, l);
    if (k >= 0) {
      const double* Dm = far[refs[k].ab].F;
      wg_add(rn, rln, Dm, rn, M, ldn);
      __syncthreads();
    }
  }
  for (int s = V.il_ptr[p]; s < V.il_ptr[p + 1]; ++s) {
    const int l = V.il_idx[s];
    if (V.chg[l] >= 0) continue;
    const int rl = V.r[l];
    const int s2 = il_slot(V, l, p);
    const double* Mo = blk_old[s2];
    double* M = V.il_blk[s2];
    const int ldo = cap_old[l], ldn = V.ilcap[l];
    wg_gemm_p(f32, rl, rn, r, 1.0, Mo, ldo, false, C.T, r > 0 ? r : 1, false, 0.0, t, rl > 0 ? rl : 1);
    wg_copy(rl, rn, t, rl > 0 ? rl : 1, M, ldn);
    const int k = find_ref(refs, C.far_begin, C.far_count, l);
    if (k >= 0) {
      const double* Dm = far[refs[k].ba].F;
      wg_add(rl, rn, Dm, rl, M, ldn);
      __syncthreads();
    }
  }
  if (has_parent) {
    double* M2M = V.arena + V.m2m_off[p];
    wg_gemm_p(f32, K, rn, r, 1.0, M2M, K, false, C.T, r > 0 ? r : 1, false, 0.0, t, K);
    wg_copy(K, rn, t, K, M2M, K);
    double* L2L = V.arena + V.l2l_off[p];
    wg_gemm_p(f32, rn, K, r, 1.0, C.S, rn > 0 ? rn : 1, false, L2L, rcp, false, 0.0, t, rn > 0 ? rn : 1);
    wg_copy(rn, K, t, rn > 0 ? rn : 1, L2L, rcp);
  }
}

// Mixed form, every rank of the level <= 32: one workgroup per changed node,
// its four waves transform the blocks of the interaction list independently
// (slot w, w + 4, ...) with FP32 matrix-core products of one 32 x 32 tile
// (v_mfma_f32_32x32x2f32; lane l holds A[l % 32][k + l / 32] and
// B[k + l / 32][l % 32], accumulator v holds D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32]);
// the intermediate S_p-side operand goes through a wave-private LDS tile.
// Every block is one tile and is read completely before it is written, which
// keeps the update correct where a block is transformed in place.
// Same arithmetic and owner rule as k_phase_b; M2M_p / L2L_p afterwards with
// the workgroup products.
__device__ inline void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// acc += A (m x k, global FP64) B (k x n, global FP64), one wave, m, n, k <= 32.
// All 16 k-steps of a lane are loaded before the first product (as FP64: a
// conversion next to its load would wait for each load in turn).
__device__ inline void wave_mm_gg(f32x16& acc, int m, int n, int k, const double* A, int lda, const double* B,
                                  int ldb) {
  const int lane = threadIdx.x & 63, i = lane & 31, kh = lane >> 5;
  double ra[16], rb[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int kk = 2 * s + kh;
    ra[s] = (i < m && kk < k) ? A[i + (int64_t)kk * lda] : 0.0;
    rb[s] = (i < n && kk < k) ? B[kk + (int64_t)i * ldb] : 0.0;
  }
#pragma unroll
  for (int s = 0; s < 16; ++s)
    if (2 * s < k) acc = __builtin_amdgcn_mfma_f32_32x32x2f32((float)ra[s], (float)rb[s], acc, 0, 0, 0);
}
// acc += A (m x k, global FP64) Bl (k x n, wave LDS tile)
__device__ inline void wave_mm_gl(f32x16& acc, int m, int n, int k, const double* A, int lda, const float (*Bl)[33]) {
  const int lane = threadIdx.x & 63, i = lane & 31, kh = lane >> 5;
  double ra[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int kk = 2 * s + kh;
    ra[s] = (i < m && kk < k) ? A[i + (int64_t)kk * lda] : 0.0;
  }
#pragma unroll
  for (int s = 0; s < 16; ++s)
    if (2 * s < k) {
      const int kk = 2 * s + kh;
      const float b = (kk < k) ? Bl[kk][i] : 0.0f;
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32((float)ra[s], b, acc, 0, 0, 0);
    }
}
__device__ inline void wave_acc_to_lds(const f32x16& acc, float (*Tl)[33]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 16; ++v) Tl[8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)][lane & 31] = acc[v];
}
// M (m x n, ld ldm) = acc + D (m x n, ld m; may be null)
__device__ inline void wave_store(const f32x16& acc, int m, int n, double* M, int ldm, const double* D) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), j = lane & 31;
    if (i < m && j < n) M[i + (int64_t)j * ldm] = (double)acc[v] + (D ? D[i + (int64_t)j * m] : 0.0);
  }
}

__global__ void __launch_bounds__(NT) k_phase_b_wave(LevelView V, int K, const Changed* chg, const FarRef* refs,
                                                     const FarPair* far, int has_parent, double* const* blk_old,
                                                     const int32_t* cap_old) {
  __shared__ float tl[4][32][33];
  const Changed C = chg[blockIdx.x];
  const int p = C.p, r = C.r, rn = C.rnew, rcp = V.rc[p];
  const int wave = threadIdx.x >> 6;
  float (*Tl)[33] = tl[wave];
  for (int s = V.il_ptr[p] + wave; s < V.il_ptr[p + 1]; s += NT / 64) {
    const int l = V.il_idx[s];
    const int rl = V.r[l], lc = V.chg[l];
    const double* Mo = blk_old[s];
    double* M = V.il_blk[s];
    const int ldo = cap_old[p], ldn = V.ilcap[p];
    const int rln = lc >= 0 ? chg[lc].rnew : rl;
    // t = M (T_l), then M = S_p t (+ D)
    f32x16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    if (lc >= 0) {
      wave_mm_gg(acc, r, rln, rl, Mo, ldo, chg[lc].T, rl > 0 ? rl : 1);
      wave_acc_to_lds(acc, Tl);
    } else {
      const int lane = threadIdx.x & 63;
      for (int e = lane; e < 32 * 32; e += 64) {
        const int i = e & 31, j = e >> 5;
        Tl[i][j] = (i < r && j < rl) ? (float)Mo[i + (int64_t)j * ldo] : 0.0f;
      }
    }
    wave_sync_lds();
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    wave_mm_gl(acc, rn, rln, r, C.S, rn > 0 ? rn : 1, Tl);
    const int k = find_ref(refs, C.far_begin, C.far_count, l);
    wave_store(acc, rn, rln, M, ldn, k >= 0 ? far[refs[k].ab].F : nullptr);
    wave_sync_lds();
    if (lc >= 0) continue;
    // block (l, p) of the unchanged l: M T_p (+ D)
    const int s2 = il_slot(V, l, p);
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    wave_mm_gg(acc, rl, rn, r, blk_old[s2], cap_old[l], C.T, r > 0 ? r : 1);
    wave_store(acc, rl, rn, V.il_blk[s2], V.ilcap[l], k >= 0 ? far[refs[k].ba].F : nullptr);
  }
  __syncthreads();
  if (has_parent) {
    double* t = C.tmp;
    double* M2M = V.arena + V.m2m_off[p];
    wg_gemm_f32(K, rn, r, 1.0, M2M, K, false, C.T, r > 0 ? r : 1, false, 0.0, t, K);
    wg_copy(K, rn, t, K, M2M, K);
    double* L2L = V.arena + V.l2l_off[p];
    wg_gemm_f32(rn, K, r, 1.0, C.S, rn > 0 ? rn : 1, false, L2L, rcp, false, 0.0, t, rn > 0 ? rn : 1);
    wg_copy(rn, K, t, rn > 0 ? rn : 1, L2L, rcp);
  }
}

// One workgroup per transformed block: kind 0 = block (p, l) of changed p, kind 1 = block
// (l, p) with l unchanged, kind 2 = M2M_p and L2L_p.  Each task brings its
// own temporary.
struct PBTask {
  int32_t chg, slot, kind, pad;
  double* t;
};
template <bool f32>
__global__ void __launch_bounds__(NT) k_phase_b_blocks(LevelView V, int K, const Changed* chg, const FarRef* refs,
                                                       const FarPair* far, const PBTask* tasks, double* const* blk_old,
                                                       const int32_t* cap_old) {
  const PBTask task = tasks[blockIdx.x];
  const Changed C = chg[task.chg];
  const int p = C.p, r = C.r, rn = C.rnew, rcp = V.rc[p];
  double* t = task.t;
  if (task.kind == 0) {
    const int s = task.slot;
    const int l = V.il_idx[s];
    const int rl = V.r[l];
    const int lc = V.chg[l];
    const double* Mo = blk_old[s];
    double* M = V.il_blk[s];
    const int ldo = cap_old[p], ldn = V.ilcap[p];
    const int rln = lc >= 0 ? chg[lc].rnew : rl;
    if (lc >= 0) wg_gemm_p(f32, r, rln, rl, 1.0, Mo, ldo, false, chg[lc].T, rl > 0 ? rl : 1, false, 0.0, t, r > 0 ? r : 1);
    else wg_copy(r, rl, Mo, ldo, t, r > 0 ? r : 1);
    wg_gemm_p(f32, rn, rln, r, 1.0, C.S, rn > 0 ? rn : 1, false, t, r > 0 ? r : 1, false, 0.0, M, ldn);
    const int k = find_ref(refs, C.far_begin, C.far_count, l);
    if (k >= 0) {
      const double* Dm = far[refs[k].ab].F;
      wg_add(rn, rln, Dm, rn, M, ldn);
    }
  } else if (task.kind == 1) {
    const int s = task.slot;  // slot of p in I_l
    const int ln = task.pad;  // the row node l of that slot
    const int rl = V.r[ln];
    const double* Mo = blk_old[s];
    double* M = V.il_blk[s];
    const int ldo = cap_old[ln], ldn = V.ilcap[ln];
    wg_gemm_p(f32, rl, rn, r, 1.0, Mo, ldo, false, C.T, r > 0 ? r : 1, false, 0.0, t, rl > 0 ? rl : 1);
    wg_copy(rl, rn, t, rl > 0 ? rl : 1, M, ldn);
    const int k = find_ref(refs, C.far_begin, C.far_count, ln);
    if (k >= 0) {
      const double* Dm = far[refs[k].ba].F;
      wg_add(rl, rn, Dm, rl, M, ldn);
    }
  } else {
    double* M2M = V.arena + V.m2m_off[p];
    wg_gemm_p(f32, K, rn, r, 1.0, M2M, K, false, C.T, r > 0 ? r : 1, false, 0.0, t, K);
    wg_copy(K, rn, t, K, M2M, K);
    double* L2L = V.arena + V.l2l_off[p];
    wg_gemm_p(f32, rn, K, r, 1.0, C.S, rn > 0 ? rn : 1, false, L2L, rcp, false, 0.0, t, rn > 0 ? rn : 1);
    wg_copy(rn, K, t, rn > 0 ? rn : 1, L2L, rcp);
  }
}

// Pointer-table updates of grown M2L blocks: before phase B the old table
// keeps the old pointer; after it both tables agree again.
struct SlotMove {
  int32_t slot, pad;
  double* ptr;
};
__global__ void __launch_bounds__(NT) k_slot_moves(double** tab, const SlotMove* mv, int count) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k < count) tab[mv[k].slot] = mv[k].ptr;
}
__global__ void __launch_bounds__(NT) k_set_caps(int32_t* cap, const int32_t* node_cap, int count) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k < count) cap[node_cap[2 * k]] = node_cap[2 * k + 1];
}

// Debug: flag any non-finite or huge (> 1e300) value in a buffer.
__global__ void __launch_bounds__(NT) k_check_finite(const double* p, int64_t n, int32_t* flag) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const double v = p[e];
    if (!(fabs(v) <= 1e300)) flag[0] = 1;
  }
}

__global__ void __launch_bounds__(NT) k_check_finite32(const float* p, int64_t n, int32_t* flag) {
  for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < n; e += (int64_t)gridDim.x * NT) {
    const float v = p[e];
    if (!(fabsf(v) <= 3e38f)) flag[0] = 1;
  }
}

__global__ void __launch_bounds__(NT) k_set_rank(int32_t* r, const Changed* chg, int nchg) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k < nchg) r[chg[k].p] = chg[k].rnew;
}

__global__ void __launch_bounds__(NT) k_set_chg(int32_t* chgidx, const Changed* chg, int nchg, int clear) {
  const int k = blockIdx.x * NT + threadIdx.x;
  if (k < nchg) chgidx[chg[k].p] = clear ? -1 : k;
}

// ------------------------------------------------------------------ top level
// Dense system of all level-2 M2L blocks (near blocks for dist <= 1).
__global__ void __launch_bounds__(NT) k_top_assemble(LevelView V, int nn, const int64_t* top_off, double* T, int ldt) {
  const int P = blockIdx.x;
  const int rP = V.r[P];
  for (int Q = 0; Q < nn; ++Q) {
    const int rQ = V.r[Q];
    if (rP == 0 || rQ == 0) continue;
    double* dst = T + top_off[P] + (int64_t)top_off[Q] * ldt;
    if (dist3(V.coord, P, Q) <= 1) wg_copy(rP, rQ, V.arena + near_block(V, P, Q), V.n[P], dst, ldt);
    else wg_copy(rP, rQ, V.il_blk[il_slot(V, P, Q)], V.ilcap[P], dst, ldt);
  }
}

// ---- dense top level: its inverse comes from the blocked LU of [T | I]
// (k_blu_*, one task), the top solve is a GEMM with it.

// C tile (64 x 64 at blockIdx) of C = alpha A B + beta C.
__global__ void __launch_bounds__(NT) k_gemm_tiles(int m, int n, int k, double alpha, const double* A, int lda, const double* B, int ldb,
                             double beta, double* C, int ldc) {
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const int mm = min(64, m - i0), nn = min(64, n - j0);
  if (mm <= 0 || nn <= 0) return;
  wg_gemm(mm, nn, k, alpha, A + i0, lda, false, B + (int64_t)j0 * ldb, ldb, false, beta, C + i0 + (int64_t)j0 * ldc,
          ldc);
}

// X (n x n) = I, grid (ceil(n / 64), ceil(n / 64)): one 64 x 64 tile each.
__global__ void __launch_bounds__(NT) k_eye(double* X, int n) {
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += NT) {
    const int i = i0 + (e & 63), j = j0 + (e >> 6);
    if (i < n && j < n) X[i + (int64_t)j * n] = i == j ? 1.0 : 0.0;
  }
}

// ------------------------------------------------------------------ solve
// Node vectors per level: X (x-part, n_i x k at xo[i] * k) and Z (z-part /
// later y-part, r_i x k at zo[i] * k); W: w_i (d x k) per elimination;
// part: partial sums of split backward tiles (64 x k per slot).
struct SolveView {
  double *X, *Z, *W, *part;
  const int64_t *xo, *zo;
  int k;
};

__global__ void __launch_bounds__(NT) k_perm_in(const double* b, int64_t ld, int k, const int64_t* perm, const int64_t* pt_begin,
                          const int32_t* n, SolveView S) {
  const int i = blockIdx.x;
  const int ni = n[i];
  double* Xi = S.X + S.xo[i] * S.k;
  if (ni > 0) WG_FOR2(ni, k, a, c) {
    Xi[a + (int64_t)c * ni] = b[perm[pt_begin[i] + a] + (int64_t)c * ld];
  }
}

__global__ void __launch_bounds__(NT) k_perm_out(double* x, int64_t ld, int k, const int64_t* perm, const int64_t* pt_begin,
                           const int32_t* n, SolveView S) {
  const int i = blockIdx.x;
  const int ni = n[i];
  const double* Xi = S.X + S.xo[i] * S.k;
  if (ni > 0) WG_FOR2(ni, k, a, c) {
    x[perm[pt_begin[i] + a] + (int64_t)c * ld] = Xi[a + (int64_t)c * ni];
  }
}

// Substitution of the eliminations (Alg. 2) with the pivot inverses stored
// explicitly: for node i with D^-1 = [[E_tt, E_tb], [E_bt, E_bb]] (blocks of
// n and r rows / columns) and G = E_tt U (the x-rows of X = D^-1 [U; 0]),
//   forward:  w = E_t. x_i (kept, n x k);  z_i += E_b. x_i;  rows of the
//             neighbours -= L w
//   backward: x_i = w - G x_nbrs + E_tb y_i
// Every step is a GEMV over 64-row tiles of one stored block: one tile per
// wave, lane = row, so each lane streams one row of the block with the
// column loads of a wave coalesced (64 consecutive rows of a column-major
// block), and the right-hand sides go through in chunks of SK columns.  The
// wave stages each 64-entry chunk of the vectors in its own LDS slice
// (entry j of the SK columns at j * SK, so one column step reads SK
// consecutive doubles that every lane shares: broadcast LDS reads, no lane
// shuffles).

// acc[c] += sign * sum_{j < cnt} A[j * lda] * x[j + c * ldx]   (c < kc, cnt <=
// 64), for the lane's row (A points at the lane's row; act: the row exists);
// xs: the wave's LDS slice of 64 * SK doubles.  The whole wave calls it.
template <int SK, typename T>
__device__ inline void wave_gemv_chunk(const T* Ag, int64_t lda, bool act, const double* xg, int64_t ldx, int cnt,
                                       int kc, int lane, double sign, double* acc, double* xs) {
  const auto A = gmem(Ag);
  const auto x = gmem(xg);
  // the previous chunk's reads of xs are ordered before these writes (LDS
  // operations of one wave complete in order), and the fences keep the
  // compiler from moving LDS accesses across the staging
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
#pragma unroll
  for (int c = 0; c < SK; ++c) xs[lane * SK + c] = (lane < cnt && c < kc) ? sign * x[lane + (int64_t)c * ldx] : 0.0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // 16 column loads in flight per wave before their products; a partial
  // chunk (cnt < 64, e.g. the blocks of leaf-level neighbours) runs whole
  // batches too, its missing columns loaded as zeros against zero vector
  // entries (the products in between are exact no-ops)
  for (int jb = 0; jb < cnt; jb += 16) {
    double av[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) av[q] = (act && jb + q < cnt) ? (double)A[(int64_t)(jb + q) * lda] : 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const double* xr = xs + (jb + q) * SK;
#pragma unroll
      for (int c = 0; c < SK; ++c) acc[c] = fma(av[q], xr[c], acc[c]);
    }
  }
}

// One segment of a tile's inner dimension, split into 64-column chunks that
// the NW waves of the workgroup take in turn (g counts chunks over segments);
// only the chunks g0 <= g < g1 are this task's.
template <int SK, int NW, typename T>
__device__ inline void seg_gemv(const T* A, int64_t lda, bool act, const double* x, int64_t ldx, int len, int kc,
                                int lane, int wave, double sign, int& g, double* acc, double* xs, int g0 = 0,
                                int g1 = INT32_MAX) {
  for (int j0 = 0; j0 < len; j0 += 64, ++g)
    if (g >= g0 && g < g1 && (g - g0) % NW == wave)
      wave_gemv_chunk<SK, T>(A + (int64_t)j0 * lda, lda, act, x + j0, ldx, min(64, len - j0), kc, lane, sign, acc,
                             xs);
}

// Sum of the waves' partial accumulators into wave 0 (returns true there).
// red[w] is also wave w's staging slice: a wave writes its partials there only
// after its last chunk, and the caller syncs before the next chunk's staging.
template <int SK, int NW>
__device__ inline bool wg_reduce_acc(double (*red)[SK][64], int lane, int wave, double* acc) {
  if (NW == 1) return true;
#pragma unroll
  for (int c = 0; c < SK; ++c) red[wave][c][lane] = acc[c];
  __syncthreads();
  if (wave != 0) return false;
#pragma unroll
  for (int c = 0; c < SK; ++c) {
    double v = 0.0;
    for (int q = 0; q < NW; ++q) v += red[q][c][lane];
    acc[c] = v;
  }
  return true;
}

// the stored L and G blocks the solve reads: FP64, or their FP32 copies
template <typename T> __device__ inline const T* solve_L(const ElimRec& R);
template <> __device__ inline const double* solve_L<double>(const ElimRec& R) { return R.L; }
template <> __device__ inline const float* solve_L<float>(const ElimRec& R) { return R.Ls; }
template <typename T> __device__ inline const T* solve_U(const ElimRec& R);
template <> __device__ inline const double* solve_U<double>(const ElimRec& R) { return R.U; }
template <> __device__ inline const float* solve_U<float>(const ElimRec& R) { return R.Us; }

// forward, step 1: w = E_t. x_i (rows < n kept in W), z_i += E_b. x_i
template <int SK, int NW, typename E>
__global__ void __launch_bounds__(64 * NW) k_solve_fwd_w(const ElimRec* recs, const STask* tasks, SolveView S) {
  __shared__ double red[NW][SK][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const STask T = tasks[blockIdx.x];
  const ElimRec R = recs[T.rec];
  const int n = R.n, r = R.r, d = R.d, k = S.k;
  const int row = T.r0 + lane;
  const bool act = row < d;
  const double* xi = S.X + S.xo[R.node] * k;
  double* wt = S.W + R.wv * k;
  double* zi = S.Z + S.zo[R.node] * k;
  for (int c0 = 0; c0 < k; c0 += SK) {
    const int kc = min(SK, k - c0);
    double acc[SK];
#pragma unroll
    for (int c = 0; c < SK; ++c) acc[c] = 0.0;
    int g = 0;
    seg_gemv<SK, NW, double>(R.lu + (act ? row : 0), d, act, xi + (int64_t)c0 * n, n, n, kc, lane, wave, 1.0, g, acc,
                             &red[wave][0][0]);
    if (wg_reduce_acc<SK, NW>(red, lane, wave, acc) && act) {
#pragma unroll
      for (int c = 0; c < SK; ++c)
        if (c < kc) {
          if (row < n) wt[row + (int64_t)(c0 + c) * n] = acc[c];
          else zi[row - n + (int64_t)(c0 + c) * r] += acc[c];
        }
    }
    if (NW > 1) __syncthreads();
  }
}

// forward, step 2: rows of the neighbours -= L w (the rows of a tile may
// belong to several neighbours; same-colour nodes share no neighbour)
template <int SK, int NW, typename E>
__global__ void __launch_bounds__(64 * NW) k_solve_fwd_upd(const ElimRec* recs, const ElimNbr* nbrs,
                                                           const STask* tasks, SolveView S) {
  __shared__ double red[NW][SK][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const STask T = tasks[blockIdx.x];
  const ElimRec R = recs[T.rec];
  const int n = R.n, k = S.k;
  const int row = T.r0 + lane;
  const bool act = row < R.M;
  double* tgt = nullptr;
  int ldt = 1;
  if (act && wave == 0)
    for (int e = 0; e < R.nnb; ++e) {
      const ElimNbr B = nbrs[R.nb_begin + e];
      if (row >= B.off && row < B.off + B.m) {
        tgt = (B.elim ? S.Z + S.zo[B.p] * k : S.X + S.xo[B.p] * k) + (row - B.off);
        ldt = B.m;
      }
    }
  const double* wt = S.W + R.wv * k;
  for (int c0 = 0; c0 < k; c0 += SK) {
    const int kc = min(SK, k - c0);
    double acc[SK];
#pragma unroll
    for (int c = 0; c < SK; ++c) acc[c] = 0.0;
    int g = 0;
    seg_gemv<SK, NW, E>(solve_L<E>(R) + (act ? row : 0), R.M, act, wt + (int64_t)c0 * n, n, n, kc, lane, wave, 1.0,
                        g, acc, &red[wave][0][0]);
    if (wg_reduce_acc<SK, NW>(red, lane, wave, acc) && tgt) {
#pragma unroll
      for (int c = 0; c < SK; ++c)
        if (c < kc) tgt[(int64_t)(c0 + c) * ldt] -= acc[c];
    }
    if (NW > 1) __syncthreads();
  }
}

// backward: x_i = w - (G x_nbrs - E_tb y_i), the inner dimension running over
// the neighbours' blocks of G and then E_tb
template <int SK, int NW, typename E>
__global__ void __launch_bounds__(64 * NW) k_solve_bwd(const ElimRec* recs, const ElimNbr* nbrs, const STask* tasks,
                                                       SolveView S) {
  __shared__ double red[NW][SK][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const STask T = tasks[blockIdx.x];
  const ElimRec R = recs[T.rec];
  const int n = R.n, r = R.r, d = R.d, k = S.k;
  const int row = T.r0 + lane;
  const bool act = row < n;
  const double* wt = S.W + R.wv * k;
  const double* yi = S.Z + S.zo[R.node] * k;
  double* xi = S.X + S.xo[R.node] * k;
  for (int c0 = 0; c0 < k; c0 += SK) {
    const int kc = min(SK, k - c0);
    double acc[SK];
#pragma unroll
    for (int c = 0; c < SK; ++c) acc[c] = 0.0;
    int g = 0;
    if constexpr (std::is_same<E, double>::value) {
      // one call site for all segments (the G blocks, then E_tb): one inlined
      // copy of the column loop keeps the register count down
      for (int q = 0; q <= R.nnb; ++q) {
        const double* Ap;
        const double* xq;
        int64_t lda;
        int len;
        double sign = 1.0;
        if (q < R.nnb) {
          const ElimNbr B = nbrs[R.nb_begin + q];
          Ap = R.U + (int64_t)B.off * n;
          lda = n;
          len = B.m;
          xq = (B.elim ? S.Z + S.zo[B.p] * k : S.X + S.xo[B.p] * k) + (int64_t)c0 * B.m;
        } else {
          Ap = R.lu + (int64_t)n * d;
          lda = d;
          len = r;
          xq = yi + (int64_t)c0 * r;
          sign = -1.0;
        }
        if (len > 0)
          seg_gemv<SK, NW, double>(Ap + (act ? row : 0), lda, act, xq, len, len, kc, lane, wave, sign, g, acc,
                                   &red[wave][0][0], T.g0, T.g1);
        if (g >= T.g1) break;  // the rest of the inner dimension belongs to later tasks
      }
    } else {
      for (int q = 0; q < R.nnb; ++q) {
        const ElimNbr B = nbrs[R.nb_begin + q];
        if (B.m == 0) continue;
        const double* xq = (B.elim ? S.Z + S.zo[B.p] * k : S.X + S.xo[B.p] * k) + (int64_t)c0 * B.m;
        seg_gemv<SK, NW, E>(solve_U<E>(R) + (act ? row : 0) + (int64_t)B.off * n, n, act, xq, B.m, B.m, kc, lane,
                            wave, 1.0, g, acc, &red[wave][0][0], T.g0, T.g1);
      }
      seg_gemv<SK, NW, double>(R.lu + (act ? row : 0) + (int64_t)n * d, d, act, yi + (int64_t)c0 * r, r, r, kc, lane,
                               wave, -1.0, g, acc, &red[wave][0][0], T.g0, T.g1);
    }
    if (wg_reduce_acc<SK, NW>(red, lane, wave, acc) && act) {
      if (T.slot < 0) {
#pragma unroll
        for (int c = 0; c < SK; ++c)
          if (c < kc) xi[row + (int64_t)(c0 + c) * n] = wt[row + (int64_t)(c0 + c) * n] - acc[c];
      } else {
#pragma unroll
        for (int c = 0; c < SK; ++c)
          if (c < kc) S.part[((int64_t)T.slot * k + c0 + c) * 64 + lane] = acc[c];
      }
    }
    if (NW > 1) __syncthreads();
  }
}

// Split backward tiles: x_i = w - (sum of the tile's partial sums, in slot
// order).  One workgroup per tile; rows over lanes, right-hand sides over the
// workgroup's waves.
__global__ void __launch_bounds__(NT) k_solve_bwd_sum(const ElimRec* recs, const SGroup* groups, SolveView S) {
  const SGroup G = groups[blockIdx.x];
  const ElimRec R = recs[G.rec];
  const int n = R.n, k = S.k;
  const int rows = min(64, n - G.r0);
  const double* wt = S.W + R.wv * k;
  double* xi = S.X + S.xo[R.node] * k;
  WG_FOR2(64, k, lr, c) {
    if (lr < rows) {
      double v = 0.0;
      for (int s = 0; s < G.ns; ++s) v += S.part[((int64_t)(G.slot0 + s) * k + c) * 64 + lr];
      const int row = G.r0 + lr;
      xi[row + (int64_t)c * n] = wt[row + (int64_t)c * n] - v;
    }
  }
}

// After the pivot solves of a colour: D^-1 = [X[:, M+r : M+r+n], X[:, M : M+r]]
// replaces the LU factors and G = X[0:n, 0:M] the U-blocks (what the solve
// reads); in the mixed form G and L go to their FP32 copies instead.  Grid
// (64-column chunks of max(d, M), records).
__global__ void __launch_bounds__(NT) k_store_solve(const ElimRec* recs) {
  const ElimRec R = recs[blockIdx.y];
  const int c0 = blockIdx.x * 64, d = R.d, n = R.n, M = R.M;
  const int nc = min(64, d - c0);
  if (nc > 0) {
    WG_FOR2(d, nc, row, cl) {
      const int c = c0 + cl;
      const int src = c < n ? M + R.r + c : M + (c - n);
      R.lu[row + (int64_t)c * d] = R.X[row + (int64_t)src * d];
    }
  }
  const int mc = min(64, M - c0);
  if (mc > 0 && n > 0) {
    if (R.Us) {
      WG_FOR2(n, mc, row, cl) {
        const int c = c0 + cl;
        R.Us[row + (int64_t)c * n] = (float)R.X[row + (int64_t)c * d];
      }
    } else {
      WG_FOR2(n, mc, row, cl) {
        const int c = c0 + cl;
        R.U[row + (int64_t)c * n] = R.X[row + (int64_t)c * d];
      }
    }
  }
  // FP32 copy of L (M x n), the chunk's columns of its n (< d) columns
  const int lc = min(64, n - c0);
  if (R.Ls && lc > 0 && M > 0) {
    WG_FOR2(M, lc, row, cl) {
      const int c = c0 + cl;
      R.Ls[row + (int64_t)c * M] = (float)R.L[row + (int64_t)c * M];
    }
  }
}

// Level change of the node vectors: x_P = [z_c ...] (up) / y_c = slices of x_P (down).
__global__ void __launch_bounds__(NT) k_vec_up(SolveView F, SolveView C, const int32_t* child_ptr, const int32_t* child,
                         const int32_t* rF, const int32_t* nC) {
  const int P = blockIdx.x;
  const int k = F.k, nP = nC[P];
  double* xP = C.X + C.xo[P] * k;
  int off = 0;
  for (int s = child_ptr[P]; s < child_ptr[P + 1]; ++s) {
    const int c = child[s], rc = rF[c];
    const double* zc = F.Z + F.zo[c] * k;
    if (rc > 0) WG_FOR2(rc, k, a, col) {
      xP[off + a + (int64_t)col * nP] = zc[a + (int64_t)col * rc];
    }
    off += rc;
  }
}

__global__ void __launch_bounds__(NT) k_vec_down(SolveView F, SolveView C, const int32_t* child_ptr, const int32_t* child,
                           const int32_t* rF, const int32_t* nC) {
  const int P = blockIdx.x;
  const int k = F.k, nP = nC[P];
  const double* xP = C.X + C.xo[P] * k;
  int off = 0;
  for (int s = child_ptr[P]; s < child_ptr[P + 1]; ++s) {
    const int c = child[s], rc = rF[c];
    double* yc = F.Z + F.zo[c] * k;
    if (rc > 0) WG_FOR2(rc, k, a, col) {
      yc[a + (int64_t)col * rc] = xP[off + a + (int64_t)col * nP];
    }
    off += rc;
  }
}

// Top solve with the explicit inverse: gather f = [z_P ...], y = Tinv f (tiled
// GEMM, separate launch), scatter y back into the z slots.
__global__ void __launch_bounds__(NT) k_top_gather(SolveView S, int nn, const int32_t* r, const int64_t* top_off, double* buf, int ldt) {
  const int P = blockIdx.x;
  const int k = S.k, rP = r[P];
  const double* z = S.Z + S.zo[P] * k;
  if (rP > 0) WG_FOR2(rP, k, a, c) buf[top_off[P] + a + (int64_t)c * ldt] = z[a + (int64_t)c * rP];
}

__global__ void __launch_bounds__(NT) k_top_scatter(SolveView S, int nn, const int32_t* r, const int64_t* top_off, const double* buf,
                              int ldt) {
  const int P = blockIdx.x;
  const int k = S.k, rP = r[P];
  double* z = S.Z + S.zo[P] * k;
  if (rP > 0) WG_FOR2(rP, k, a, c) z[a + (int64_t)c * rP] = buf[top_off[P] + a + (int64_t)c * ldt];
}

// ------------------------------------------------------------------ BD preconditioner
// Block-diagonal preconditioner (Sec. 4.3): the dense diagonal block of every
// box of level l_BD, inverted by the blocked LU path.  Assembly: box b's block
// D (n_b x n_b, points [pt_begin[b], pt_begin[b + 1]) in tree order) and the
// identity in X; grid (64-column chunks, boxes).
__global__ void __launch_bounds__(NT) k_bd_assemble(const double* pts, const double* w, const double* diag,
                                                    const int64_t* pt_begin, const BluTask* tasks) {
  const BluTask t = tasks[blockIdx.y];
  const int nb = t.d, c0 = blockIdx.x * 64;
  if (threadIdx.x == 0 && blockIdx.x == 0) *t.info = 0;
  if (c0 >= nb) return;
  const int nc = min(64, nb - c0);
  const int64_t p0 = pt_begin[blockIdx.y];
  WG_FOR2(nb, nc, a, cl) {
    const int b = c0 + cl;
    double v;
    if (a == b) {
      v = diag[p0 + a];
    } else {
      const double* x = pts + 3 * (p0 + a);
      const double* y = pts + 3 * (p0 + b);
      const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
      v = w[p0 + b] / (4.0 * M_PI * sqrt(dx * dx + dy * dy + dz * dz));
    }
    t.lu[a + (int64_t)b * nb] = v;
    t.X[a + (int64_t)b * nb] = a == b ? 1.0 : 0.0;
  }
}

// z_b = D_b^-1 r_b for every box (one workgroup each), in the caller's point
// order (perm: tree position -> original index).
__global__ void __launch_bounds__(NT) k_bd_apply(const BluTask* tasks, const int64_t* pt_begin, const int64_t* perm,
                                                 const double* r, double* z) {
  __shared__ double rb[BD_MAXN];
  const BluTask t = tasks[blockIdx.x];
  const int nb = t.d;
  const int64_t p0 = pt_begin[blockIdx.x];
  for (int j = threadIdx.x; j < nb; j += NT) rb[j] = r[perm[p0 + j]];
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += NT) {
    double acc = 0.0;
    for (int j = 0; j < nb; ++j) acc += t.X[i + (int64_t)j * nb] * rb[j];
    z[perm[p0 + i]] = acc;
  }
}

}  // namespace ifmm
