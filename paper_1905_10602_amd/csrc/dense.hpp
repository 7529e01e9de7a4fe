// Workgroup-level dense FP64 linear algebra for gfx950 (256 threads = 4 wave64).
//
// All matrices are column-major with an explicit leading dimension and live
// in global memory (L2-resident for the sizes the IFMM produces).  Every
// routine is called by all threads of the workgroup and ends with a barrier,
// so results are visible to the whole workgroup on return.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ifmm {

constexpr int NT = 256;           // threads per workgroup
constexpr int JAC_MAXPAIR = 1024;  // Jacobi eigen-solver handles n <= 2048

// C(m x n) = alpha * op(A) * op(B) + beta * C, op = transpose if tA / tB.
// op(A) is m x k, op(B) is k x n.  beta == 0 overwrites C (NaNs in C ignored).
// LDS tiles of 64 x 16 (A) and 16 x 64 (B); each thread owns a 4 x 4 block
// of the 64 x 64 output tile, rows strided by 16 for coalesced stores.
__device__ inline void wg_gemm(int m, int n, int k, double alpha, const double* A, int lda, bool tA,
                               const double* B, int ldb, bool tB, double beta, double* C, int ldc) {
  __shared__ double sA[16][65];
  __shared__ double sB[16][65];
  const int tid = threadIdx.x;
  const int tr = tid & 15, tc = tid >> 4;
  for (int i0 = 0; i0 < m; i0 += 64) {
    for (int j0 = 0; j0 < n; j0 += 64) {
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
      for (int k0 = 0; k0 < k; k0 += 16) {
        // load A tile: rows i0..i0+63, cols k0..k0+15  (64*16 = 1024 values, 4 per thread)
        for (int e = tid; e < 1024; e += NT) {
          int ii, kk;
          if (!tA) { ii = e & 63; kk = e >> 6; } else { kk = e & 15; ii = e >> 4; }
          const int gi = i0 + ii, gk = k0 + kk;
          double v = 0.0;
          if (gi < m && gk < k) v = tA ? A[gk + (int64_t)gi * lda] : A[gi + (int64_t)gk * lda];
          sA[kk][ii] = v;
        }
        for (int e = tid; e < 1024; e += NT) {
          int kk, jj;
          if (!tB) { kk = e & 15; jj = e >> 4; } else { jj = e & 63; kk = e >> 6; }
          const int gk = k0 + kk, gj = j0 + jj;
          double v = 0.0;
          if (gk < k && gj < n) v = tB ? B[gj + (int64_t)gk * ldb] : B[gk + (int64_t)gj * ldb];
          sB[kk][jj] = v;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
          double av[4], bv[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) av[a] = sA[kk][tr + 16 * a];
#pragma unroll
          for (int b = 0; b < 4; ++b) bv[b] = sB[kk][tc + 16 * b];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int gj = j0 + tc + 16 * b;
        if (gj >= n) continue;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int gi = i0 + tr + 16 * a;
          if (gi >= m) continue;
          double* c = C + gi + (int64_t)gj * ldc;
          *c = (beta == 0.0) ? alpha * acc[a][b] : fma(alpha, acc[a][b], beta * (*c));
        }
      }
    }
  }
  __syncthreads();
}

// dst(m x n) = alpha * src
__device__ inline void wg_copy(int m, int n, const double* src, int lds, double* dst, int ldd, double alpha = 1.0) {
  const int64_t tot = (int64_t)m * n;
  for (int64_t e = threadIdx.x; e < tot; e += NT) {
    const int i = (int)(e % m), j = (int)(e / m);
    dst[i + (int64_t)j * ldd] = alpha * src[i + (int64_t)j * lds];
  }
  __syncthreads();
}

__device__ inline void wg_fill(int m, int n, double* dst, int ldd, double v) {
  const int64_t tot = (int64_t)m * n;
  for (int64_t e = threadIdx.x; e < tot; e += NT) {
    const int i = (int)(e % m), j = (int)(e / m);
    dst[i + (int64_t)j * ldd] = v;
  }
  __syncthreads();
}

// In-place LU with partial pivoting (row interchanges), A = P L U, L unit
// lower.  piv[j] = row swapped with row j at step j (0-based).  The pivot is
// the entry of largest magnitude, the first one on ties.  Returns (to every
// thread) the first step with an exactly zero pivot + 1, or 0.
__device__ inline int wg_getrf(int d, double* A, int lda, int32_t* piv) {
  __shared__ double sv[NT];
  __shared__ int si[NT];
  __shared__ int s_info;
  if (threadIdx.x == 0) s_info = 0;
  __syncthreads();
  const int tid = threadIdx.x;
  for (int j = 0; j < d; ++j) {
    double best = -1.0;
    int bi = d;
    for (int i = j + tid; i < d; i += NT) {
      const double v = fabs(A[i + (int64_t)j * lda]);
      if (v > best) { best = v; bi = i; }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
      if (tid < s) {
        const double v2 = sv[tid + s];
        const int i2 = si[tid + s];
        if (v2 > sv[tid] || (v2 == sv[tid] && i2 < si[tid])) { sv[tid] = v2; si[tid] = i2; }
      }
      __syncthreads();
    }
    const int p = si[0];
    const double pv = sv[0];
    __syncthreads();
    if (tid == 0) {
      piv[j] = p;
      if (pv == 0.0 && s_info == 0) s_info = j + 1;
    }
    if (p != j) {
      for (int c = tid; c < d; c += NT) {
        const double t = A[j + (int64_t)c * lda];
        A[j + (int64_t)c * lda] = A[p + (int64_t)c * lda];
        A[p + (int64_t)c * lda] = t;
      }
    }
    __syncthreads();
    const double dj = A[j + (int64_t)j * lda];
    if (dj != 0.0) {
      const double inv = 1.0 / dj;
      for (int i = j + 1 + tid; i < d; i += NT) A[i + (int64_t)j * lda] *= inv;
    }
    __syncthreads();
    const int rem = d - j - 1;
    const int64_t tot = (int64_t)rem * rem;
    for (int64_t e = tid; e < tot; e += NT) {
      const int i = j + 1 + (int)(e % rem), c = j + 1 + (int)(e / rem);
      A[i + (int64_t)c * lda] -= A[i + (int64_t)j * lda] * A[j + (int64_t)c * lda];
    }
    __syncthreads();
  }
  const int info = s_info;
  __syncthreads();
  return info;
}

// Solves (P L U) X = B in place for B (d x nc), with the factors of wg_getrf.
__device__ inline void wg_getrs(int d, const double* LU, int lda, const int32_t* piv, double* B, int ldb, int nc) {
  const int tid = threadIdx.x;
  // row interchanges, in order
  for (int c = tid; c < nc; c += NT) {
    for (int j = 0; j < d; ++j) {
      const int p = piv[j];
      if (p != j) {
        const double t = B[j + (int64_t)c * ldb];
        B[j + (int64_t)c * ldb] = B[p + (int64_t)c * ldb];
        B[p + (int64_t)c * ldb] = t;
      }
    }
  }
  __syncthreads();
  // forward: unit lower
  for (int j = 0; j < d - 1; ++j) {
    const int rem = d - j - 1;
    const int64_t tot = (int64_t)rem * nc;
    for (int64_t e = tid; e < tot; e += NT) {
      const int i = j + 1 + (int)(e % rem), c = (int)(e / rem);
      B[i + (int64_t)c * ldb] -= LU[i + (int64_t)j * lda] * B[j + (int64_t)c * ldb];
    }
    __syncthreads();
  }
  // backward: upper
  for (int j = d - 1; j >= 0; --j) {
    const double djj = LU[j + (int64_t)j * lda];
    for (int c = tid; c < nc; c += NT) B[j + (int64_t)c * ldb] /= djj;
    __syncthreads();
    const int64_t tot = (int64_t)j * nc;
    for (int64_t e = tid; e < tot; e += NT) {
      const int i = (int)(e % j), c = (int)(e / j);
      B[i + (int64_t)c * ldb] -= LU[i + (int64_t)j * lda] * B[j + (int64_t)c * ldb];
    }
    __syncthreads();
  }
}

// Symmetric eigen-decomposition by the cyclic Jacobi method with a parallel
// (round-robin) ordering: A (n x n, overwritten) = V diag(lam) V^T.  On return
// lam is sorted in descending order and V holds the matching eigenvectors.
// Vtmp (n x n) is workspace.
__device__ inline void wg_syev_jacobi(int n, double* A, int lda, double* V, int ldv, double* Vtmp, double* lam) {
  // one entry per rotation pair of a round: n <= 2 * JAC_MAXPAIR
  __shared__ double s_c[JAC_MAXPAIR], s_s[JAC_MAXPAIR];
  __shared__ int s_p[JAC_MAXPAIR], s_q[JAC_MAXPAIR];
  __shared__ double s_red[NT];
  __shared__ int s_stop;
  const int tid = threadIdx.x;
  // Vtmp = I
  for (int64_t e = tid; e < (int64_t)n * n; e += NT) {
    const int i = (int)(e % n), j = (int)(e / n);
    Vtmp[i + (int64_t)j * n] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int m = (n + 1) & ~1;  // players, one dummy if n is odd
  const int npair = m / 2;
  // rotations stop once every off-diagonal entry is below 1e-17 ||A||_F
  // (absolute accuracy of order u ||A|| for every eigenvalue)
  {
    double fro = 0.0;
    for (int64_t e = tid; e < (int64_t)n * n; e += NT) {
      const int i = (int)(e % n), j = (int)(e / n);
      const double v = A[i + (int64_t)j * lda];
      fro += v * v;
    }
    s_red[tid] = fro;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
      if (tid < s) s_red[tid] += s_red[tid + s];
      __syncthreads();
    }
  }
  const double tol = 1e-17 * sqrt(s_red[0]);
  __syncthreads();
  for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
    if (tid == 0) s_stop = 1;
    __syncthreads();
    for (int round = 0; round < m - 1; ++round) {
      // round-robin pairing: player m-1 fixed, others rotate
      for (int k = tid; k < npair; k += NT) {
        int a, b;
        if (k == 0) { a = m - 1; b = round; }
        else { a = (round + k) % (m - 1); b = (round - k + (m - 1)) % (m - 1); }
        int p = a < b ? a : b, q = a < b ? b : a;
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p + (int64_t)q * lda];
          const double app = A[p + (int64_t)p * lda], aqq = A[q + (int64_t)q * lda];
          if (fabs(apq) > tol) {
            s_stop = 0;
            const double theta = (aqq - app) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        } else {
          q = -1;
        }
        s_p[k] = p; s_q[k] = q; s_c[k] = c; s_s[k] = s;
      }
      __syncthreads();
      // rows: A <- J^T A   (rows p, q)
      for (int64_t e = tid; e < (int64_t)npair * n; e += NT) {
        const int k = (int)(e % npair), j = (int)(e / npair);
        const int q = s_q[k];
        if (q < 0 || s_s[k] == 0.0) continue;
        const int p = s_p[k];
        const double c = s_c[k], s = s_s[k];
        const double x = A[p + (int64_t)j * lda], y = A[q + (int64_t)j * lda];
        A[p + (int64_t)j * lda] = c * x - s * y;
        A[q + (int64_t)j * lda] = s * x + c * y;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int64_t e = tid; e < (int64_t)npair * n; e += NT) {
        const int k = (int)(e % npair), i = (int)(e / npair);
        const int q = s_q[k];
        if (q < 0 || s_s[k] == 0.0) continue;
        const int p = s_p[k];
        const double c = s_c[k], s = s_s[k];
        double x = A[i + (int64_t)p * lda], y = A[i + (int64_t)q * lda];
        A[i + (int64_t)p * lda] = c * x - s * y;
        A[i + (int64_t)q * lda] = s * x + c * y;
        x = Vtmp[i + (int64_t)p * n];
        y = Vtmp[i + (int64_t)q * n];
        Vtmp[i + (int64_t)p * n] = c * x - s * y;
        Vtmp[i + (int64_t)q * n] = s * x + c * y;
      }
      __syncthreads();
      // exact zeros on the rotated off-diagonal entries
      for (int k = tid; k < npair; k += NT) {
        const int q = s_q[k];
        if (q < 0 || s_s[k] == 0.0) continue;
        const int p = s_p[k];
        A[p + (int64_t)q * lda] = 0.0;
        A[q + (int64_t)p * lda] = 0.0;
      }
      __syncthreads();
    }
    if (s_stop) break;
    __syncthreads();
  }
  // sort descending (ties by index) and permute eigenvectors
  for (int j = tid; j < n; j += NT) {
    const double v = A[j + (int64_t)j * lda];
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double u = A[i + (int64_t)i * lda];
      if (u > v || (u == v && i < j)) ++rank;
    }
    lam[rank] = v;
    for (int i = 0; i < n; ++i) V[i + (int64_t)rank * ldv] = Vtmp[i + (int64_t)j * n];
  }
  __syncthreads();
}

}  // namespace ifmm
