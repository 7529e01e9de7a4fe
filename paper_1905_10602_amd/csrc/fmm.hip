// Black-box (Chebyshev) FMM matrix-vector product and the right-preconditioned
// FGMRES of the FMBEM driver, on the device.
//
// Alg. 4 of the paper: build the FMM tree, precompute P2M, M2M, M2L, L2L, L2P
// and P2P, then run GMRES from x = 0 with the preconditioner of Alg. 5 (the
// IFMM solve, or none).  Sec. 4.2 lets that FMM differ from the one the IFMM
// is built on; here it is the Chebyshev FMM of Fong and Darve on the same
// uniform octree (root cube and depth rule), with its own interpolation order.
//
// Matrix-vector product y = A~ x, all levels >= 2:
//   upward    m_leaf = S diag(w) x_leaf;  m_P = sum_c M2M_c m_c
//   transfer  l_t = (1 / h_l) sum_{s in I_t} U_{off(t,s)} m_s
//             (U: unit-size M2L per box offset, K(x, y) homogeneous of degree -1)
//   downward  l_c += M2M_c^T l_P
//   leaves    y = S^T l_leaf + sum_{q in N_i + {i}} P2P_iq x_q
// The transfer step is a batched GEMM: the (target, source) pairs of a level
// are grouped by offset, their source multipoles gathered into contiguous
// columns, and every group of <= 64 pairs multiplied by its U in one
// workgroup; a per-target reduction (fixed order) adds the partial results,
// so the product is deterministic.
//
// FGMRES (Saad): right preconditioning with the preconditioned directions
// kept, classical Gram-Schmidt applied twice, Givens rotations on the host;
// the stopping test uses the recurrence residual |g_{j+1}| / ||b||.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "cheb.hpp"
#include "dense.hpp"
#include "engine.hpp"
#include "fmm.hpp"

namespace ifmm {

#define FCHK(x)                                                    \
  do {                                                             \
    hipError_t e_ = (x);                                           \
    if (e_ != hipSuccess) {                                        \
      err = std::string(#x) + " failed: " + hipGetErrorString(e_); \
      return -3;                                                   \
    }                                                              \
  } while (0)

static double fnow() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ operators
// Unit-side M2L for box offsets d in [-3, 3]^3 (d = source - target):
//   U_d[m, m'] = 1 / (4 pi |xb_m / 2 - d - xb_m' / 2|) for side 1 (scaled by 1/side).
__global__ void __launch_bounds__(NT) k_fmm_m2l_ops(int nc, double* out) {
  const int o = blockIdx.x;
  const int dx = o % 7 - 3, dy = (o / 7) % 7 - 3, dz = o / 49 - 3;
  const int K = nc * nc * nc;
  double* U = out + (int64_t)o * K * K;
  const bool near = abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1;
  WG_FOR2(K, K, m, mp) {
    double v = 0.0;
    if (!near) {
      const double x = 0.5 * (cheb_node(nc, m % nc) - cheb_node(nc, mp % nc)) - dx;
      const double y = 0.5 * (cheb_node(nc, (m / nc) % nc) - cheb_node(nc, (mp / nc) % nc)) - dy;
      const double z = 0.5 * (cheb_node(nc, m / (nc * nc)) - cheb_node(nc, mp / (nc * nc))) - dz;
      v = 1.0 / (4.0 * M_PI * sqrt(x * x + y * y + z * z));
    }
    U[m + (int64_t)mp * K] = v;
  }
}

// M2M of a child in octant o (bit e set: upper half along axis e), parent frame.
__global__ void __launch_bounds__(NT) k_fmm_m2m_ops(int nc, double* out) {
  const int o = blockIdx.x;
  const int K = nc * nc * nc;
  double* M = out + (int64_t)o * K * K;
  const double sx = (o & 1) ? 0.5 : -0.5, sy = (o & 2) ? 0.5 : -0.5, sz = (o & 4) ? 0.5 : -0.5;
  WG_FOR2(K, K, m, mp) {
    const double x = sx + 0.5 * cheb_node(nc, mp % nc);
    const double y = sy + 0.5 * cheb_node(nc, (mp / nc) % nc);
    const double z = sz + 0.5 * cheb_node(nc, mp / (nc * nc));
    M[m + (int64_t)mp * K] = cheb_S(nc, m % nc, x) * cheb_S(nc, (m / nc) % nc, y) * cheb_S(nc, m / (nc * nc), z);
  }
}

// Leaf interpolation weights S[m, j] = S(xb_m, y_j) (K x n_leaf per leaf, at pt_begin * K).
__global__ void __launch_bounds__(NT) k_fmm_leaf_S(int nc, const double* pts, const int64_t* pt_begin, const int32_t* coord,
                             const double* lo, double side, double* S) {
  const int i = blockIdx.x;
  const int K = nc * nc * nc;
  const int64_t b = pt_begin[i];
  const int n = (int)(pt_begin[i + 1] - b);
  const double h = 0.5 * side;
  double c[3];
  for (int e = 0; e < 3; ++e) c[e] = lo[e] + ((double)coord[3 * i + e] + 0.5) * side;
  double* Si = S + b * K;
  if (n > 0) WG_FOR2(K, n, m, j) {
    const double* p = pts + 3 * (b + j);
    Si[m + (int64_t)j * K] = cheb_S(nc, m % nc, (p[0] - c[0]) / h) * cheb_S(nc, (m / nc) % nc, (p[1] - c[1]) / h) *
                             cheb_S(nc, m / (nc * nc), (p[2] - c[2]) / h);
  }
}

// ------------------------------------------------------------------ matvec
__global__ void __launch_bounds__(NT) k_fmm_perm_in(const double* x, const int64_t* perm, double* xs, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (t < n) xs[t] = x[perm[t]];
}

__global__ void __launch_bounds__(NT) k_fmm_perm_out(const double* ys, const int64_t* perm, double* y, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (t < n) y[perm[t]] = ys[t];
}

// m_leaf = S diag(w) x_leaf; one workgroup per leaf, leaf_base = global index of leaf 0
__global__ void __launch_bounds__(NT) k_fmm_p2m(int K, const double* S, const int64_t* pt_begin, const double* w, const double* xs,
                          double* mult, int64_t leaf_base) {
  const int i = blockIdx.x;
  const int64_t b = pt_begin[i];
  const int n = (int)(pt_begin[i + 1] - b);
  const double* Si = S + b * K;
  double* mi = mult + (leaf_base + i) * K;
  for (int m = threadIdx.x; m < K; m += NT) {
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc += Si[m + (int64_t)j * K] * (w[b + j] * xs[b + j]);
    mi[m] = acc;
  }
}

// m_P = sum_c M2M_oct(c) m_c; one workgroup per parent (global index base + blockIdx.x)
__global__ void __launch_bounds__(NT) k_fmm_m2m(int K, const double* m2m, const int32_t* child_ptr, const int32_t* child,
                          const int32_t* oct, double* mult, int64_t base) {
  __shared__ double sm[216];  // K <= 216, one output row per thread
  const int64_t P = base + blockIdx.x;
  const int m = threadIdx.x;
  double acc = 0.0;
  for (int e = child_ptr[P]; e < child_ptr[P + 1]; ++e) {
    const int c = child[e];
    __syncthreads();
    for (int q = threadIdx.x; q < K; q += NT) sm[q] = mult[(int64_t)c * K + q];
    __syncthreads();
    const double* M = m2m + (int64_t)oct[c] * K * K;
    if (m < K)
      for (int q = 0; q < K; ++q) acc += M[m + (int64_t)q * K] * sm[q];
  }
  if (m < K) mult[P * K + m] = acc;
}

// gathered source multipoles of the pairs: G[:, p] = m_{src(p)}
__global__ void __launch_bounds__(NT) k_fmm_gather(int K, const int32_t* src, const double* mult, double* G, int64_t npairs) {
  const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (e >= npairs * K) return;
  const int64_t p = e / K;
  const int m = (int)(e - p * K);
  G[e] = mult[(int64_t)src[p] * K + m];
}

// partial[:, start:start+count] = U_off G[:, start:start+count]
__global__ void __launch_bounds__(NT) k_fmm_m2l(int K, const FmmHandle::GemmTask* tasks, const double* m2l, const double* G,
                          double* part) {
  const FmmHandle::GemmTask t = tasks[blockIdx.x];
  wg_gemm(K, t.count, K, 1.0, m2l + (int64_t)t.off * K * K, K, false, G + t.start * K, K, false, 0.0,
          part + t.start * K, K);
}

// l_t = (1/h) sum_pairs partial + M2M_oct(t)^T l_parent (levels > 2); one
// workgroup per target node of the level (global index base + blockIdx.x)
__global__ void __launch_bounds__(NT) k_fmm_local(int K, const int64_t* tp_ptr, const int64_t* tp, const double* part, double inv_h,
                            const double* m2m, const int32_t* oct, const int32_t* par, double* loc, int64_t base,
                            int has_parent) {
  __shared__ double sl[216];
  const int64_t t = base + blockIdx.x;
  const int m = threadIdx.x;
  if (has_parent) {
    const int P = par[t];
    for (int q = threadIdx.x; q < K; q += NT) sl[q] = loc[(int64_t)P * K + q];
  }
  __syncthreads();
  if (m >= K) return;
  double acc = 0.0;
  for (int64_t e = tp_ptr[t]; e < tp_ptr[t + 1]; ++e) acc += part[tp[e] * K + m];
  acc *= inv_h;
  if (has_parent) {
    const double* M = m2m + (int64_t)oct[t] * K * K;
    double a2 = 0.0;
    for (int q = 0; q < K; ++q) a2 += M[q + (int64_t)m * K] * sl[q];
    acc += a2;
  }
  loc[t * K + m] = acc;
}

// y_leaf = S^T l_leaf + near field; one workgroup per leaf, 4 lanes per target
// point split the sources; sources staged through LDS one neighbour at a time
__global__ void __launch_bounds__(NT) k_fmm_leaf_eval(int K, const double* S, const int64_t* pt_begin, const int32_t* nbr_ptr,
                                const int32_t* nbr, const double* pts, const double* w, const double* diag,
                                const double* xs, const double* loc, int64_t leaf_base, double* ys) {
  __shared__ double sl[216];
  __shared__ double sp[4][256];
  __shared__ double red[NT];
  const int i = blockIdx.x;
  const int64_t b = pt_begin[i];
  const int n = (int)(pt_begin[i + 1] - b);
  for (int q = threadIdx.x; q < K; q += NT) sl[q] = loc[(leaf_base + i) * K + q];
  __syncthreads();
  const double* Si = S + b * K;
  for (int j0 = 0; j0 < n; j0 += NT / 4) {
    const int jl = j0 + (threadIdx.x >> 2), part = threadIdx.x & 3;
    const bool act = jl < n;
    double acc = 0.0, px = 0, py = 0, pz = 0;
    if (act) {
      for (int m = part; m < K; m += 4) acc += Si[m + (int64_t)jl * K] * sl[m];
      px = pts[3 * (b + jl)]; py = pts[3 * (b + jl) + 1]; pz = pts[3 * (b + jl) + 2];
    }
    for (int e = nbr_ptr[i] - 1; e < nbr_ptr[i + 1]; ++e) {
      const int q = e < nbr_ptr[i] ? i : nbr[e];
      const int64_t qb = pt_begin[q];
      const int nq = (int)(pt_begin[q + 1] - qb);
      for (int k0 = 0; k0 < nq; k0 += 256) {
        const int kc = min(256, nq - k0);
        __syncthreads();
        for (int k = threadIdx.x; k < kc; k += NT) {
          const int64_t g = qb + k0 + k;
          sp[0][k] = pts[3 * g]; sp[1][k] = pts[3 * g + 1]; sp[2][k] = pts[3 * g + 2];
          sp[3][k] = w[g] * xs[g];
        }
        __syncthreads();
        if (act)
          for (int k = part; k < kc; k += 4) {
            const int64_t g = qb + k0 + k;
            if (g == b + jl) {
              acc += diag[g] * xs[g];
            } else {
              const double dx = px - sp[0][k], dy = py - sp[1][k], dz = pz - sp[2][k];
              acc += sp[3][k] / (4.0 * M_PI * sqrt(dx * dx + dy * dy + dz * dz));
            }
          }
      }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (act && part == 0) ys[b + jl] = red[threadIdx.x] + red[threadIdx.x + 1] + red[threadIdx.x + 2] + red[threadIdx.x + 3];
    __syncthreads();
  }
}

// ------------------------------------------------------------------ GMRES vector kernels
// partial dot products of w with columns 0..nv-1 of V (ld n): grid (chunks, nv)
__global__ void __launch_bounds__(NT) k_gm_dots(const double* V, int64_t n, const double* w, int64_t chunk, double* part) {
  const int64_t a = (int64_t)blockIdx.x * chunk, bnd = (n < a + chunk) ? n : a + chunk;
  const double* v = V + (int64_t)blockIdx.y * n;
  double s = 0.0;
  for (int64_t e = a + threadIdx.x; e < bnd; e += NT) s += v[e] * w[e];
  const double tot = wg_sum(s);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = tot;
}

__global__ void __launch_bounds__(NT) k_gm_dots_fin(const double* part, int nchunk, double* out) {
  double s = 0.0;
  for (int e = threadIdx.x; e < nchunk; e += NT) s += part[(int64_t)blockIdx.x * nchunk + e];
  const double tot = wg_sum(s);
  if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

// w -= V[:, 0:nv] h  (h on device, nv <= 1024)
__global__ void __launch_bounds__(NT) k_gm_sub(const double* V, int64_t n, int nv, const double* h, double* w) {
  __shared__ double sh[1024];
  for (int e = threadIdx.x; e < nv; e += NT) sh[e] = h[e];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i >= n) return;
  double s = w[i];
  for (int j = 0; j < nv; ++j) s -= V[i + (int64_t)j * n] * sh[j];
  w[i] = s;
}

// y = a x + b y
__global__ void __launch_bounds__(NT) k_gm_axpby(int64_t n, double a, const double* x, double b, double* y) {
  const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (i < n) y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

// ------------------------------------------------------------------ host
template <class T>
static int up(T** d, const std::vector<T>& v, hipStream_t s, std::string& err) {
  FCHK(hipMalloc((void**)d, std::max<size_t>(v.size(), 1) * sizeof(T)));
  if (!v.empty()) FCHK(hipMemcpyAsync(*d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  FCHK(hipStreamSynchronize(s));
  return 0;
}

int fmm_setup(FmmHandle& h, const double* pts, int64_t n, const double* w, const double* diag, double diag_scalar,
              std::string& err) {
  err = h.tree.build(pts, n, h.leaf_max, 3);
  if (!err.empty()) return -1;
  err = h.tree.coincident(pts);
  if (!err.empty()) return -1;
  {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
      err = "no HIP device";
      return -3;
    }
  }
  h.N = n;
  h.K = h.nc * h.nc * h.nc;
  const int K = h.K;
  const Tree& T = h.tree;
  const int D = T.depth;
  FCHK(hipGetDevice(&h.device));
  if (!h.stream) {
    // a blocking stream: ordered with the null stream, on which callers
    // (torch's default stream among them) produce the device vectors
    FCHK(hipStreamCreate(&h.stream));
    h.own_stream = true;
  }
  // points, weights, diagonal in tree order
  std::vector<double> P(3 * n), W(n), Dg(n);
  for (int64_t t = 0; t < n; ++t) {
    const int64_t p = T.perm[t];
    for (int e = 0; e < 3; ++e) P[3 * t + e] = pts[3 * p + e];
    W[t] = w ? w[p] : 1.0;
    Dg[t] = diag ? diag[p] : diag_scalar;
    if (!std::isfinite(W[t]) || !std::isfinite(Dg[t])) {
      err = "non-finite weight or diagonal entry";
      return -5;
    }
  }
  // global node numbering over levels 2..D
  h.node_base.assign(D + 2, 0);
  int64_t nodes = 0;
  for (int l = 2; l <= D; ++l) {
    h.node_base[l] = nodes;
    nodes += T.levels[l].n;
  }
  h.node_base[D + 1] = nodes;
  h.nodes = nodes;
  std::vector<int32_t> oct(nodes, 0), par(nodes, -1), cptr(nodes + 1, 0), chl, nlev(nodes, 0);
  for (int l = 2; l <= D; ++l) {
    const Level& L = T.levels[l];
    for (int i = 0; i < L.n; ++i) {
      const int64_t g = h.node_base[l] + i;
      oct[g] = (L.coord[3 * i] & 1) | ((L.coord[3 * i + 1] & 1) << 1) | ((L.coord[3 * i + 2] & 1) << 2);
      par[g] = l > 2 ? (int32_t)(h.node_base[l - 1] + L.parent[i]) : -1;
      nlev[g] = l;
    }
  }
  for (int l = 2; l <= D; ++l) {
    const Level& L = T.levels[l];
    for (int i = 0; i < L.n; ++i) {
      const int64_t g = h.node_base[l] + i;
      cptr[g] = (int32_t)chl.size();
      if (l < D)
        for (int e = L.child_ptr[i]; e < L.child_ptr[i + 1]; ++e) chl.push_back((int32_t)(h.node_base[l + 1] + L.child[e]));
    }
  }
  cptr[nodes] = (int32_t)chl.size();
  // M2L pairs grouped by (level, offset), then GEMM tasks of <= 64 pairs
  std::vector<int32_t> src;
  std::vector<std::vector<int64_t>> tpl(nodes);
  h.tasks.clear();
  for (int l = 2; l <= D; ++l) {
    const Level& L = T.levels[l];
    std::vector<std::vector<std::pair<int32_t, int32_t>>> byoff(343);
    for (int t = 0; t < L.n; ++t)
      for (int e = L.il_ptr[t]; e < L.il_ptr[t + 1]; ++e) {
        const int s = L.il[e];
        const int dx = L.coord[3 * s] - L.coord[3 * t], dy = L.coord[3 * s + 1] - L.coord[3 * t + 1],
                  dz = L.coord[3 * s + 2] - L.coord[3 * t + 2];
        if (std::abs(dx) > 3 || std::abs(dy) > 3 || std::abs(dz) > 3) {
          err = "interaction-list offset outside [-3, 3]^3";
          return -6;
        }
        byoff[(dx + 3) + 7 * ((dy + 3) + 7 * (dz + 3))].push_back({t, s});
      }
    for (int o = 0; o < 343; ++o) {
      const auto& v = byoff[o];
      for (size_t a = 0; a < v.size(); a += 64) {
        FmmHandle::GemmTask gt;
        gt.off = o;
        gt.count = (int32_t)std::min<size_t>(64, v.size() - a);
        gt.start = (int64_t)src.size() + (int64_t)a;
        h.tasks.push_back(gt);
      }
      for (const auto& ts : v) {
        tpl[h.node_base[l] + ts.first].push_back((int64_t)src.size());
        src.push_back((int32_t)(h.node_base[l] + ts.second));
      }
    }
  }
  h.npairs = (int64_t)src.size();
  std::vector<int64_t> tptr(nodes + 1, 0), tp;
  tp.reserve(h.npairs);
  for (int64_t g = 0; g < nodes; ++g) {
    tptr[g] = (int64_t)tp.size();
    tp.insert(tp.end(), tpl[g].begin(), tpl[g].end());
  }
  tptr[nodes] = (int64_t)tp.size();
  h.flops_m2l = 2.0 * K * K * (double)h.npairs;
  // leaves
  const Level& LF = T.levels[D];
  std::vector<int64_t> ptb(LF.n + 1);
  for (int i = 0; i < LF.n; ++i) ptb[i] = LF.pt_begin[i];
  ptb[LF.n] = n;
  int rc;
  std::vector<int64_t> perm(T.perm.begin(), T.perm.end());
  if ((rc = up(&h.d_pts, P, h.stream, err))) return rc;
  if ((rc = up(&h.d_w, W, h.stream, err))) return rc;
  if ((rc = up(&h.d_diag, Dg, h.stream, err))) return rc;
  if ((rc = up(&h.d_perm, perm, h.stream, err))) return rc;
  if ((rc = up(&h.d_pt_begin, ptb, h.stream, err))) return rc;
  if ((rc = up(&h.d_leaf_coord, LF.coord, h.stream, err))) return rc;
  if ((rc = up(&h.d_nbr_ptr, LF.nbr_ptr, h.stream, err))) return rc;
  if ((rc = up(&h.d_nbr, LF.nbr, h.stream, err))) return rc;
  if ((rc = up(&h.d_node_oct, oct, h.stream, err))) return rc;
  if ((rc = up(&h.d_node_par, par, h.stream, err))) return rc;
  if ((rc = up(&h.d_child_ptr, cptr, h.stream, err))) return rc;
  if ((rc = up(&h.d_child, chl, h.stream, err))) return rc;
  if ((rc = up(&h.d_tp_ptr, tptr, h.stream, err))) return rc;
  if ((rc = up(&h.d_tp, tp, h.stream, err))) return rc;
  if ((rc = up(&h.d_pair_src, src, h.stream, err))) return rc;
  if ((rc = up(&h.d_tasks, h.tasks, h.stream, err))) return rc;
  std::vector<double> lo(T.lo, T.lo + 3);
  double* d_lo = nullptr;
  if ((rc = up(&d_lo, lo, h.stream, err))) return rc;
  FCHK(hipMalloc((void**)&h.d_S, (size_t)K * n * 8));
  FCHK(hipMalloc((void**)&h.d_m2m, (size_t)8 * K * K * 8));
  FCHK(hipMalloc((void**)&h.d_m2l, (size_t)343 * K * K * 8));
  FCHK(hipMalloc((void**)&h.d_mult, (size_t)nodes * K * 8));
  FCHK(hipMalloc((void**)&h.d_loc, (size_t)nodes * K * 8));
  FCHK(hipMalloc((void**)&h.d_gath, (size_t)std::max<int64_t>(h.npairs, 1) * K * 8));
  FCHK(hipMalloc((void**)&h.d_part, (size_t)std::max<int64_t>(h.npairs, 1) * K * 8));
  FCHK(hipMalloc((void**)&h.d_xs, (size_t)n * 8));
  FCHK(hipMalloc((void**)&h.d_ys, (size_t)n * 8));
  const double side = 2.0 * T.H / (double)(1 << D);
  hipLaunchKernelGGL(k_fmm_leaf_S, dim3(LF.n), dim3(NT), 0, h.stream, h.nc, h.d_pts, h.d_pt_begin, h.d_leaf_coord,
                     d_lo, side, h.d_S);
  hipLaunchKernelGGL(k_fmm_m2m_ops, dim3(8), dim3(NT), 0, h.stream, h.nc, h.d_m2m);
  hipLaunchKernelGGL(k_fmm_m2l_ops, dim3(343), dim3(NT), 0, h.stream, h.nc, h.d_m2l);
  FCHK(hipGetLastError());
  FCHK(hipStreamSynchronize(h.stream));
  FCHK(hipFree(d_lo));
  return 0;
}

int fmm_apply(FmmHandle& h, const double* x, double* y, std::string& err) {
  const double t0 = fnow();
  const Tree& T = h.tree;
  const int D = T.depth, K = h.K;
  const int64_t n = h.N;
  const unsigned g1 = (unsigned)((n + NT - 1) / NT);
  hipLaunchKernelGGL(k_fmm_perm_in, dim3(g1), dim3(NT), 0, h.stream, x, h.d_perm, h.d_xs, n);
  hipLaunchKernelGGL(k_fmm_p2m, dim3(T.levels[D].n), dim3(NT), 0, h.stream, K, h.d_S, h.d_pt_begin, h.d_w, h.d_xs,
                     h.d_mult, h.node_base[D]);
  for (int l = D - 1; l >= 2; --l)
    hipLaunchKernelGGL(k_fmm_m2m, dim3(T.levels[l].n), dim3(NT), 0, h.stream, K, h.d_m2m, h.d_child_ptr, h.d_child,
                       h.d_node_oct, h.d_mult, h.node_base[l]);
  if (h.npairs > 0) {
    const int64_t ne = h.npairs * K;
    hipLaunchKernelGGL(k_fmm_gather, dim3((unsigned)((ne + NT - 1) / NT)), dim3(NT), 0, h.stream, K, h.d_pair_src,
                       h.d_mult, h.d_gath, h.npairs);
    hipLaunchKernelGGL(k_fmm_m2l, dim3((unsigned)h.tasks.size()), dim3(NT), 0, h.stream, K, h.d_tasks, h.d_m2l,
                       h.d_gath, h.d_part);
  }
  for (int l = 2; l <= D; ++l) {
    const double half = T.H / (double)(1 << l);
    hipLaunchKernelGGL(k_fmm_local, dim3(T.levels[l].n), dim3(NT), 0, h.stream, K, h.d_tp_ptr, h.d_tp, h.d_part,
                       1.0 / (2.0 * half), h.d_m2m, h.d_node_oct, h.d_node_par, h.d_loc, h.node_base[l], l > 2 ? 1 : 0);
  }
  hipLaunchKernelGGL(k_fmm_leaf_eval, dim3(T.levels[D].n), dim3(NT), 0, h.stream, K, h.d_S, h.d_pt_begin, h.d_nbr_ptr,
                     h.d_nbr, h.d_pts, h.d_w, h.d_diag, h.d_xs, h.d_loc, h.node_base[D], h.d_ys);
  hipLaunchKernelGGL(k_fmm_perm_out, dim3(g1), dim3(NT), 0, h.stream, h.d_ys, h.d_perm, y, n);
  FCHK(hipGetLastError());
  FCHK(hipStreamSynchronize(h.stream));
  h.matvecs++;
  h.t_matvec += fnow() - t0;
  return 0;
}

int fmm_gmres(FmmHandle& h, Handle* pre, const double* b, double* x, double tol, int restart, int maxit, int* iters,
              double* relres, std::string& err, BdHandle* bd) {
  const int64_t n = h.N;
  const int m = restart;
  const int64_t chunk = 1 << 15;
  const int nchunk = (int)((n + chunk - 1) / chunk);
  // V (n x (m+1)), Z (n x m), w, r, partials, dots
  const int64_t need = (n * (2 * m + 3) + (int64_t)nchunk * (m + 2) + 2 * (m + 2) + 64) * 8;
  if (need > h.gm_bytes) {
    if (h.d_gm) FCHK(hipFree(h.d_gm));
    h.d_gm = nullptr;
    h.gm_bytes = 0;
    FCHK(hipMalloc((void**)&h.d_gm, (size_t)need));
    h.gm_bytes = need;
  }
  double* V = h.d_gm;
  double* Z = V + n * (m + 1);
  double* w = Z + n * m;
  double* r = w + n;
  double* part = r + n;
  double* dots = part + (int64_t)nchunk * (m + 2);
  const unsigned g1 = (unsigned)((n + NT - 1) / NT);
  hipStream_t s = h.stream;
  std::vector<double> hd(m + 2);
  auto dotv = [&](const double* Vb, int nv, const double* v, std::string& e2) -> int {
    hipLaunchKernelGGL(k_gm_dots, dim3(nchunk, nv), dim3(NT), 0, s, Vb, n, v, chunk, part);
    hipLaunchKernelGGL(k_gm_dots_fin, dim3(nv), dim3(NT), 0, s, part, nchunk, dots);
    hipError_t e = hipMemcpyAsync(hd.data(), dots, nv * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      e2 = std::string("GMRES reduction failed: ") + hipGetErrorString(e);
      return -3;
    }
    return 0;
  };
  auto precond = [&](const double* v, double* z, std::string& e2) -> int {
    if (bd) {
      hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        e2 = std::string("stream sync failed: ") + hipGetErrorString(e);
        return -3;
      }
      return bd_apply(*bd, v, z, e2);
    }
    if (!pre) {
      hipLaunchKernelGGL(k_gm_axpby, dim3(g1), dim3(NT), 0, s, n, 1.0, v, 0.0, z);
      return 0;
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      e2 = std::string("stream sync failed: ") + hipGetErrorString(e);
      return -3;
    }
    return solve(*pre, v, z, 1, n, 1, e2);
  };
  int rc;
  hipLaunchKernelGGL(k_gm_axpby, dim3(g1), dim3(NT), 0, s, n, 0.0, b, 0.0, x);  // x = 0
  if ((rc = dotv(b, 1, b, err))) return rc;
  const double bnorm = std::sqrt(hd[0]);
  *iters = 0;
  *relres = 0.0;
  if (bnorm == 0.0) return 0;
  int its = 0;
  double rr = 1.0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  while (its < maxit) {
    // r = b - A x
    if (its == 0) {
      hipLaunchKernelGGL(k_gm_axpby, dim3(g1), dim3(NT), 0, s, n, 1.0, b, 0.0, r);
    } else {
      if ((rc = fmm_apply(h, x, w, err))) return rc;
      hipLaunchKernelGGL(k_gm_axpby, dim3(g1), dim3(NT), 0, s, n, 1.0, b, 0.0, r);
      hipLaunchKernelGGL(k_gm_axpby, dim3(g1), dim3(NT), 0, s, n, -1.0, w, 1.0, r);
    }
    if ((rc = dotv(r, 1, r, err))) return rc;
    const double beta = std::sqrt(hd[0]);
    rr = beta / bnorm;
    if (rr <= tol) break;
    const int mm = std::min(m, maxit - its);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    hipLaunchKernelGGL(k_gm_axpby, dim3(g1), dim3(NT), 0, s, n, 1.0 / beta, r, 0.0, V);
    int k = 0;
    for (int j = 0; j < mm; ++j) {
      double* vj = V + (int64_t)j * n;
      double* zj = Z + (int64_t)j * n;
      if ((rc = precond(vj, zj, err))) return rc;
      if ((rc = fmm_apply(h, zj, w, err))) return rc;
      // CGS2
      double* hc = &H[(size_t)j * (m + 1)];
      for (int pass = 0; pass < 2; ++pass) {
        if ((rc = dotv(V, j + 1, w, err))) return rc;  // the coefficients stay in dots on the device
        hipLaunchKernelGGL(k_gm_sub, dim3(g1), dim3(NT), 0, s, V, n, j + 1, dots, w);
        for (int i = 0; i <= j; ++i) hc[i] += hd[i];
      }
      if ((rc = dotv(w, 1, w, err))) return rc;
      const double hn = std::sqrt(hd[0]);
      hc[j + 1] = hn;
      if (hn > 0.0) hipLaunchKernelGGL(k_gm_axpby, dim3(g1), dim3(NT), 0, s, n, 1.0 / hn, w, 0.0, V + (int64_t)(j + 1) * n);
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * hc[i] + sn[i] * hc[i + 1];
        hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
        hc[i] = t;
      }
      const double a = hc[j], bb = hc[j + 1];
      if (bb == 0.0) {
        cs[j] = a >= 0.0 ? 1.0 : -1.0;
        sn[j] = 0.0;
      } else {
        const double rad = std::hypot(a, bb);
        cs[j] = a / rad;
        sn[j] = bb / rad;
      }
      hc[j] = cs[j] * a + sn[j] * bb;
      hc[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      ++its;
      rr = std::fabs(g[j + 1]) / bnorm;
      if (rr <= tol || hc[j] == 0.0) break;
    }
    // y = R^-1 g, x += Z y
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int c = i + 1; c < k; ++c) t -= H[(size_t)c * (m + 1) + i] * y[c];
      y[i] = t / H[(size_t)i * (m + 1) + i];
    }
    for (int i = 0; i < k; ++i) y[i] = -y[i];
    FCHK(hipMemcpyAsync(dots, y.data(), k * 8, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_gm_sub, dim3(g1), dim3(NT), 0, s, Z, n, k, dots, x);
    FCHK(hipStreamSynchronize(s));
    if (rr <= tol) break;
  }
  FCHK(hipGetLastError());
  FCHK(hipStreamSynchronize(s));
  *iters = its;
  *relres = rr;
  return 0;
}

void fmm_release(FmmHandle& h) {
  void* ptrs[] = {h.d_pts, h.d_w, h.d_diag, h.d_perm, h.d_pt_begin, h.d_leaf_coord, h.d_nbr_ptr, h.d_nbr,
                  h.d_node_oct, h.d_node_par, h.d_child_ptr, h.d_child, h.d_tp_ptr, h.d_tp, h.d_pair_src,
                  h.d_tasks, h.d_S, h.d_m2m, h.d_m2l, h.d_mult, h.d_loc, h.d_gath, h.d_part, h.d_xs, h.d_ys,
                  h.d_gm};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (h.own_stream && h.stream) (void)hipStreamDestroy(h.stream);
  h.stream = nullptr;
}

}  // namespace ifmm
