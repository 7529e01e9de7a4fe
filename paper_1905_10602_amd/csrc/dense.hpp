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

// The same address as a global-memory pointer.  Pointers read from task
// tables are generic to the compiler, and generic (flat) loads count against
// the LDS counter as well, so a wait for an LDS result also waits for every
// global load in flight; loads through these pointers are global loads.
template <class T>
__device__ inline const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ inline __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
// Global-memory pointer when G (the operands of the GEMM tiles), else the
// generic pointer (a caller whose operands may live in LDS).
template <bool G, class T>
__device__ inline auto gsel(T* p) {
  if constexpr (G) return gmem(p);
  else return p;
}

// Workgroup-strided loop over an R x C index range, rows fastest (coalesced
// for column-major data).  One 32-bit division at entry, none per step.
// Requires R > 0.
#define WG_FOR2(R, C, i, c)                                                                          \
  for (int i = (int)(threadIdx.x % (unsigned)(R)), c = (int)(threadIdx.x / (unsigned)(R)),           \
           i##_di = (int)((unsigned)NT % (unsigned)(R)), i##_dc = (int)((unsigned)NT / (unsigned)(R)); \
       c < (C); i += i##_di, c += i##_dc, (i >= (R) ? (i -= (R), ++c) : 0))

// Small product (m, n, k <= 32): both operands staged whole in LDS (the
// caller's buffer of at least 2 * 32 * 33 doubles), one pass, no k-chunks.
template <bool G = true>
__device__ inline void wg_gemm_small(int m, int n, int k, double alpha, const double* A_, int lda, bool tA,
                                     const double* B_, int ldb, bool tB, double beta, double* C_, int ldc,
                                     double* smem) {
  const auto A = gsel<G>(A_);
  const auto B = gsel<G>(B_);
  const auto C = gsel<G>(C_);
  const int tid = threadIdx.x;
  double (*As)[33] = reinterpret_cast<double (*)[33]>(smem);
  double (*Bs)[33] = reinterpret_cast<double (*)[33]>(smem + 32 * 33);
  for (int e = tid; e < m * k; e += NT) {
    const int i = e % m, q = e / m;
    As[i][q] = tA ? A[q + (int64_t)i * lda] : A[i + (int64_t)q * lda];
  }
  for (int e = tid; e < k * n; e += NT) {
    const int q = e % k, j = e / k;
    Bs[q][j] = tB ? B[j + (int64_t)q * ldb] : B[q + (int64_t)j * ldb];
  }
  __syncthreads();
  for (int e = tid; e < m * n; e += NT) {
    const int i = e % m, j = e / m;
    double acc = 0.0;
    for (int q = 0; q < k; ++q) acc = fma(As[i][q], Bs[q][j], acc);
    auto c = C + i + (int64_t)j * ldc;
    *c = (beta == 0.0) ? alpha * acc : fma(alpha, acc, beta * (*c));
  }
  __syncthreads();
}

// C(m x n) = alpha * op(A) * op(B) + beta * C, op = transpose if tA / tB.
// op(A) is m x k, op(B) is k x n.  beta == 0 overwrites C (NaNs in C ignored).
// LDS tiles of 64 x 16 (A) and 16 x 64 (B); each thread owns a 4 x 4 block
// of the 64 x 64 output tile, rows strided by 16 for coalesced stores.
template <bool G = true>
__device__ inline void wg_gemm(int m, int n, int k, double alpha, const double* A_, int lda, bool tA,
                               const double* B_, int ldb, bool tB, double beta, double* C_, int ldc) {
  const auto A = gsel<G>(A_);
  const auto B = gsel<G>(B_);
  const auto C = gsel<G>(C_);
  __shared__ double smem[2 * 16 * 65 + 64];
  double (*sA)[65] = reinterpret_cast<double (*)[65]>(smem);
  double (*sB)[65] = reinterpret_cast<double (*)[65]>(smem + 16 * 65);
  const int tid = threadIdx.x;
  if (m <= 32 && n <= 32 && k <= 32) {
    wg_gemm_small<G>(m, n, k, alpha, A_, lda, tA, B_, ldb, tB, beta, C_, ldc, smem);
    return;
  }
  const int tr = tid & 15, tc = tid >> 4;
  for (int i0 = 0; i0 < m; i0 += 64) {
    for (int j0 = 0; j0 < n; j0 += 64) {
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
      // the next k-chunk is fetched into registers while the current one is
      // multiplied out of LDS (4 A and 4 B values per thread)
      double ra[4], rb[4];
      auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * NT;
          int ii, kk;
          if (!tA) { ii = e & 63; kk = e >> 6; } else { kk = e & 15; ii = e >> 4; }
          const int gi = i0 + ii, gk = k0 + kk;
          ra[q] = (gi < m && gk < k) ? (tA ? A[gk + (int64_t)gi * lda] : A[gi + (int64_t)gk * lda]) : 0.0;
          int kb, jb;
          if (!tB) { kb = e & 15; jb = e >> 4; } else { jb = e & 63; kb = e >> 6; }
          const int gk2 = k0 + kb, gj = j0 + jb;
          rb[q] = (gk2 < k && gj < n) ? (tB ? B[gj + (int64_t)gk2 * ldb] : B[gk2 + (int64_t)gj * ldb]) : 0.0;
        }
      };
      auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * NT;
          int ii, kk;
          if (!tA) { ii = e & 63; kk = e >> 6; } else { kk = e & 15; ii = e >> 4; }
          sA[kk][ii] = ra[q];
          int kb, jb;
          if (!tB) { kb = e & 15; jb = e >> 4; } else { jb = e & 63; kb = e >> 6; }
          sB[kb][jb] = rb[q];
        }
      };
      if (k > 0) {
        fetch(0);
        stash();
      }
      __syncthreads();
      for (int k0 = 0; k0 < k; k0 += 16) {
        const bool more = k0 + 16 < k;
        if (more) fetch(k0 + 16);
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
        if (more) stash();
        __syncthreads();
      }
      // epilogue: every C value loaded, then combined, then stored (a wait
      // for a load issued after a store also waits for the store)
      double cv[4][4];
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int gi = i0 + tr + 16 * a, gj = j0 + tc + 16 * b;
          cv[a][b] = (beta != 0.0 && gi < m && gj < n) ? C[gi + (int64_t)gj * ldc] : 0.0;
        }
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int a = 0; a < 4; ++a) cv[a][b] = (beta == 0.0) ? alpha * acc[a][b] : fma(alpha, acc[a][b], beta * cv[a][b]);
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int gi = i0 + tr + 16 * a, gj = j0 + tc + 16 * b;
          if (gi < m && gj < n) C[gi + (int64_t)gj * ldc] = cv[a][b];
        }
    }
  }
  __syncthreads();
}

// The same product with FP32 matrix cores: operands rounded to FP32 on their
// way into LDS, FP32 accumulation (v_mfma_f32_32x32x2f32), the result
// combined with C in FP64.  Each of the four waves owns a 32 x 32 quadrant of
// the 64 x 64 output tile (formed transposed, B^T A^T, so that each lane owns
// rows of C).  Operand lane layout of the 32x32x2 instruction:
// lane l holds A[l % 32][l / 32] and B[l / 32][l % 32]; accumulator register
// v of lane l holds D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].
typedef float f32x16 __attribute__((ext_vector_type(16)));
// 64 x 64 tiles, k-chunks of 16 through one LDS buffer pair (lds: at least
// 2 x 16 x 68 floats), the next chunk prefetched into registers.
template <bool G = true>
__device__ inline void wg_gemm_f32_lite(int m, int n, int k, double alpha, const double* A_, int lda, bool tA,
                                        const double* B_, int ldb, bool tB, double beta, double* C_, int ldc,
                                        float* lds) {
  const auto A = gsel<G>(A_);
  const auto B = gsel<G>(B_);
  const auto C = gsel<G>(C_);
  float (*fA)[68] = reinterpret_cast<float (*)[68]>(lds);
  float (*fB)[68] = reinterpret_cast<float (*)[68]>(lds + 16 * 68);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  for (int i0 = 0; i0 < m; i0 += 64) {
    for (int j0 = 0; j0 < n; j0 += 64) {
      f32x16 acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
      // prefetched as FP64 and converted when stashed: a conversion next to
      // its load would wait for each load in turn
      double ra[4], rb[4];
      auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * NT;
          int ii, kk;
          if (!tA) { ii = e & 63; kk = e >> 6; } else { kk = e & 15; ii = e >> 4; }
          const int gi = i0 + ii, gk = k0 + kk;
          ra[q] = (gi < m && gk < k) ? (tA ? A[gk + (int64_t)gi * lda] : A[gi + (int64_t)gk * lda]) : 0.0;
          int kb, jb;
          if (!tB) { kb = e & 15; jb = e >> 4; } else { jb = e & 63; kb = e >> 6; }
          const int gk2 = k0 + kb, gj = j0 + jb;
          rb[q] = (gk2 < k && gj < n) ? (tB ? B[gj + (int64_t)gk2 * ldb] : B[gk2 + (int64_t)gj * ldb]) : 0.0;
        }
      };
      auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * NT;
          int ii, kk;
          if (!tA) { ii = e & 63; kk = e >> 6; } else { kk = e & 15; ii = e >> 4; }
          fA[kk][ii] = (float)ra[q];
          int kb, jb;
          if (!tB) { kb = e & 15; jb = e >> 4; } else { jb = e & 63; kb = e >> 6; }
          fB[kb][jb] = (float)rb[q];
        }
      };
      if (k > 0) {
        fetch(0);
        stash();
      }
      __syncthreads();
      for (int k0 = 0; k0 < k; k0 += 16) {
        const bool more = k0 + 16 < k;
        if (more) fetch(k0 + 16);
        // transposed product (B^T A^T): lane l holds rows l % 32 of C
#pragma unroll
        for (int kk = 0; kk < 16; kk += 2) {
          const float a = fA[kk + (lane >> 5)][wr + (lane & 31)];
          const float b = fB[kk + (lane >> 5)][wc + (lane & 31)];
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(b, a, acc, 0, 0, 0);
        }
        __syncthreads();
        if (more) stash();
        __syncthreads();
      }
      const int gi = i0 + wr + (lane & 31);
      if (gi < m) {
        // every C value loaded, then combined, then stored
        double cv[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int gj = j0 + wc + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          cv[v] = (beta != 0.0 && gj < n) ? C[gi + (int64_t)gj * ldc] : 0.0;
        }
#pragma unroll
        for (int v = 0; v < 16; ++v)
          cv[v] = (beta == 0.0) ? alpha * (double)acc[v] : fma(alpha, (double)acc[v], beta * cv[v]);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int gj = j0 + wc + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          if (gj < n) C[gi + (int64_t)gj * ldc] = cv[v];
        }
      }
    }
  }
  __syncthreads();
}

// 64 x 64 tiles, k-chunks of 32 through two LDS buffer pairs (lds: at least
// 2 x 2 x 32 x 65 floats): chunk c + 1 is loaded into registers while chunk c
// is multiplied, then written to the other pair; one barrier per chunk.  Rows
// padded to 65 floats (conflict-free column writes).  For long inner dimensions.
template <bool G = true>
__device__ inline void wg_gemm_f32_kc32(int m, int n, int k, double alpha, const double* A_, int lda, bool tA,
                                        const double* B_, int ldb, bool tB, double beta, double* C_, int ldc,
                                        float* lds) {
  const auto A = gsel<G>(A_);
  const auto B = gsel<G>(B_);
  const auto C = gsel<G>(C_);
  constexpr int KC = 32;
  float (*fA)[KC][65] = reinterpret_cast<float (*)[KC][65]>(lds);
  float (*fB)[KC][65] = reinterpret_cast<float (*)[KC][65]>(lds + 2 * KC * 65);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  for (int i0 = 0; i0 < m; i0 += 64) {
    for (int j0 = 0; j0 < n; j0 += 64) {
      f32x16 acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
      double ra[8], rb[8];
      auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int e = tid + q * NT;
          int ii, kk;
          if (!tA) { ii = e & 63; kk = e >> 6; } else { kk = e & 31; ii = e >> 5; }
          const int gi = i0 + ii, gk = k0 + kk;
          ra[q] = (gi < m && gk < k) ? (tA ? A[gk + (int64_t)gi * lda] : A[gi + (int64_t)gk * lda]) : 0.0;
          int kb, jb;
          if (!tB) { kb = e & 31; jb = e >> 5; } else { jb = e & 63; kb = e >> 6; }
          const int gk2 = k0 + kb, gj = j0 + jb;
          rb[q] = (gk2 < k && gj < n) ? (tB ? B[gj + (int64_t)gk2 * ldb] : B[gk2 + (int64_t)gj * ldb]) : 0.0;
        }
      };
      auto stash = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int e = tid + q * NT;
          int ii, kk;
          if (!tA) { ii = e & 63; kk = e >> 6; } else { kk = e & 31; ii = e >> 5; }
          fA[buf][kk][ii] = (float)ra[q];
          int kb, jb;
          if (!tB) { kb = e & 31; jb = e >> 5; } else { jb = e & 63; kb = e >> 6; }
          fB[buf][kb][jb] = (float)rb[q];
        }
      };
      if (k > 0) {
        fetch(0);
        stash(0);
      }
      __syncthreads();
      int buf = 0;
      for (int k0 = 0; k0 < k; k0 += KC) {
        const bool more = k0 + KC < k;
        if (more) fetch(k0 + KC);
#pragma unroll
        for (int kk = 0; kk < KC; kk += 2) {
          const float a = fA[buf][kk + (lane >> 5)][wr + (lane & 31)];
          const float b = fB[buf][kk + (lane >> 5)][wc + (lane & 31)];
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(b, a, acc, 0, 0, 0);
        }
        if (more) stash(buf ^ 1);
        __syncthreads();
        buf ^= 1;
      }
      const int gi = i0 + wr + (lane & 31);
      if (gi < m) {
        // every C value loaded, then combined, then stored
        double cv[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int gj = j0 + wc + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          cv[v] = (beta != 0.0 && gj < n) ? C[gi + (int64_t)gj * ldc] : 0.0;
        }
#pragma unroll
        for (int v = 0; v < 16; ++v)
          cv[v] = (beta == 0.0) ? alpha * (double)acc[v] : fma(alpha, (double)acc[v], beta * cv[v]);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int gj = j0 + wc + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          if (gj < n) C[gi + (int64_t)gj * ldc] = cv[v];
        }
      }
    }
  }
  __syncthreads();
}

// FP32 matrix-core product with the lite tile; one LDS buffer serves it and
// the small FP64 product.
__device__ inline void wg_gemm_f32(int m, int n, int k, double alpha, const double* A, int lda, bool tA,
                                   const double* B, int ldb, bool tB, double beta, double* C, int ldc) {
  __shared__ double lbuf[2 * 32 * 33];  // >= 2 x 16 x 68 floats
  if (m <= 32 && n <= 32 && k <= 32) {  // too small for matrix cores: the FP64 one-pass product
    wg_gemm_small(m, n, k, alpha, A, lda, tA, B, ldb, tB, beta, C, ldc, lbuf);
    return;
  }
  wg_gemm_f32_lite(m, n, k, alpha, A, lda, tA, B, ldb, tB, beta, C, ldc, reinterpret_cast<float*>(lbuf));
}

// The same for kernels whose products have long inner dimensions: k >= 96
// takes the double-buffered tile (more LDS and registers, hence its own
// kernel instances), shorter ones the lite tile in the same buffer.
__device__ inline void wg_gemm_f32_deep(int m, int n, int k, double alpha, const double* A, int lda, bool tA,
                                        const double* B, int ldb, bool tB, double beta, double* C, int ldc) {
  __shared__ double lbuf[2 * 32 * 65];  // 2 x 2 x 32 x 65 floats
  if (m <= 32 && n <= 32 && k <= 32) {
    wg_gemm_small(m, n, k, alpha, A, lda, tA, B, ldb, tB, beta, C, ldc, lbuf);
    return;
  }
  if (k < 96) wg_gemm_f32_lite(m, n, k, alpha, A, lda, tA, B, ldb, tB, beta, C, ldc, reinterpret_cast<float*>(lbuf));
  else wg_gemm_f32_kc32(m, n, k, alpha, A, lda, tA, B, ldb, tB, beta, C, ldc, reinterpret_cast<float*>(lbuf));
}

// FP64 matrix-core product C = alpha op(A) B + beta C (op(A) m x k, A^T when
// tA; B k x n; column major), v_mfma_f64_16x16x4f64, 64 x 64 output tiles per
// workgroup with k-chunks of 16 staged through LDS (the next chunk prefetched
// into registers), each wave a 32 x 32 quarter as 2 x 2 blocks of 16 x 16.
// The product is formed transposed, C^T = B^T A^T, so that the accumulator
// of lane l, register v, holds C[l % 16][4 v + l / 16] of its block: 16
// consecutive rows of C per column, coalesced.  Lane layout of the
// instruction (checked on the device): lane l supplies a = P[l % 16][l / 16]
// and b = Q[l / 16][l % 16] of D = P Q and receives D[4 v + l / 16][l % 16]
// in register v; here P = B^T and Q = A^T.  Per 1024 multiply-adds a wave
// reads 1 KB of operands from LDS, against 4 KB for the FMA tile's 4 x 4
// register blocks, which makes this tile bound by the matrix cores rather
// than by LDS bandwidth.
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <bool G = true>
__device__ inline void wg_gemm_f64m(int m, int n, int k, double alpha, const double* A_, int lda, const double* B_,
                                    int ldb, double beta, double* C_, int ldc, bool tA = false) {
  const auto A = gsel<G>(A_);
  const auto B = gsel<G>(B_);
  const auto C = gsel<G>(C_);
  __shared__ double lds64[2 * 16 * 68];  // >= 2 x 32 x 33 for the small product
  if (m <= 32 && n <= 32 && k <= 32) {   // too small for the tiles: the one-pass product
    wg_gemm_small<G>(m, n, k, alpha, A_, lda, tA, B_, ldb, false, beta, C_, ldc, lds64);
    return;
  }
  double (*fA)[68] = reinterpret_cast<double (*)[68]>(lds64);
  double (*fB)[68] = reinterpret_cast<double (*)[68]>(lds64 + 16 * 68);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  for (int i0 = 0; i0 < m; i0 += 64) {
    for (int j0 = 0; j0 < n; j0 += 64) {
      f64x4 acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
      double ra[4], rb[4];
      // chunk k0..k0+15: A rows i0 + (e & 63), column k0 + (e >> 6) (A
      // transposed: k0 + (e & 15) of column i0 + (e >> 4)); B rows k0 + (e & 15),
      // column j0 + (e >> 4); e = tid + 256 q
      auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * NT;
          const int ii = tA ? e >> 4 : e & 63, kk = tA ? e & 15 : e >> 6;
          const int gi = i0 + ii, gk = k0 + kk;
          ra[q] = (gi < m && gk < k) ? (tA ? A[gk + (int64_t)gi * lda] : A[gi + (int64_t)gk * lda]) : 0.0;
          const int kb = e & 15, jb = e >> 4;
          const int gk2 = k0 + kb, gj = j0 + jb;
          rb[q] = (gk2 < k && gj < n) ? B[gk2 + (int64_t)gj * ldb] : 0.0;
        }
      };
      auto stash = [&]() {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + q * NT;
          if (tA) fA[e & 15][e >> 4] = ra[q];
          else fA[e >> 6][e & 63] = ra[q];
          fB[e & 15][e >> 4] = rb[q];
        }
      };
      if (k > 0) {
        fetch(0);
        stash();
      }
      __syncthreads();
      for (int k0 = 0; k0 < k; k0 += 16) {
        const bool more = k0 + 16 < k;
        if (more) fetch(k0 + 16);
#pragma unroll
        for (int ks = 0; ks < 16; ks += 4) {
          const int kr = ks + lk;
          const double a0 = fA[kr][wr + lr], a1 = fA[kr][wr + 16 + lr];
          const double b0 = fB[kr][wc + lr], b1 = fB[kr][wc + 16 + lr];
          // block (row half ri, column half cj): a-operand from B, b-operand from A
          acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a0, acc[0][0], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(b0, a1, acc[1][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a0, acc[0][1], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(b1, a1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
        if (more) stash();
        __syncthreads();
      }
      // acc[ri][cj] register v of lane l: C[i0 + wr + 16 ri + l % 16][j0 + wc + 16 cj + 4 v + l / 16]
      // every C value loaded, then combined, then stored (a wait for a load
      // issued after a store also waits for the store)
      double cv[2][2][4];
#pragma unroll
      for (int ri = 0; ri < 2; ++ri)
#pragma unroll
        for (int cj = 0; cj < 2; ++cj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = i0 + wr + 16 * ri + lr, j = j0 + wc + 16 * cj + 4 * v + lk;
            cv[ri][cj][v] = (beta != 0.0 && i < m && j < n) ? C[i + (int64_t)j * ldc] : 0.0;
          }
#pragma unroll
      for (int ri = 0; ri < 2; ++ri)
#pragma unroll
        for (int cj = 0; cj < 2; ++cj)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            cv[ri][cj][v] = beta == 0.0 ? alpha * acc[ri][cj][v] : fma(alpha, acc[ri][cj][v], beta * cv[ri][cj][v]);
#pragma unroll
      for (int ri = 0; ri < 2; ++ri)
#pragma unroll
        for (int cj = 0; cj < 2; ++cj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = i0 + wr + 16 * ri + lr, j = j0 + wc + 16 * cj + 4 * v + lk;
            if (i < m && j < n) C[i + (int64_t)j * ldc] = cv[ri][cj][v];
          }
    }
  }
  __syncthreads();
}

// precision switch of the Schur-complement and basis-change products
__device__ inline void wg_gemm_p(bool f32, int m, int n, int k, double alpha, const double* A, int lda, bool tA,
                                 const double* B, int ldb, bool tB, double beta, double* C, int ldc) {
  if (f32) wg_gemm_f32(m, n, k, alpha, A, lda, tA, B, ldb, tB, beta, C, ldc);
  else wg_gemm(m, n, k, alpha, A, lda, tA, B, ldb, tB, beta, C, ldc);
}

// Element-wise pass over an R x C index range (rows fastest, the order of
// WG_FOR2), EW_B elements per thread at a time: ld(i, c) for all of them
// (the loads), then st(i, c, value) (the arithmetic and the stores).  A wait
// for a load issued after a store also waits for that store, so a loop that
// loads and stores one element at a time pays a memory latency per element.
// No barrier at the end.
constexpr int EW_B = 8;
template <class Ld, class St>
__device__ inline void wg_each2(int R, int C, Ld ld, St st) {
  if (R <= 0 || C <= 0) return;
  const int di = (int)((unsigned)NT % (unsigned)R), dc = (int)((unsigned)NT / (unsigned)R);
  int i = (int)(threadIdx.x % (unsigned)R), c = (int)(threadIdx.x / (unsigned)R);
  while (c < C) {
    int ri[EW_B], ci[EW_B];
    decltype(ld(0, 0)) v[EW_B];
#pragma unroll
    for (int q = 0; q < EW_B; ++q) {
      ri[q] = i;
      ci[q] = c;
      i += di;
      c += dc;
      if (i >= R) {
        i -= R;
        ++c;
      }
    }
#pragma unroll
    for (int q = 0; q < EW_B; ++q)
      if (ci[q] < C) v[q] = ld(ri[q], ci[q]);
#pragma unroll
    for (int q = 0; q < EW_B; ++q)
      if (ci[q] < C) st(ri[q], ci[q], v[q]);
  }
}

// dst(m x n) = alpha * src (global memory, no overlap)
__device__ inline void wg_copy(int m, int n, const double* src, int lds, double* dst, int ldd, double alpha = 1.0) {
  const auto S = gmem(src);
  const auto D = gmem(dst);
  wg_each2(m, n, [&](int i, int j) { return S[i + (int64_t)j * lds]; },
           [&](int i, int j, double v) { D[i + (int64_t)j * ldd] = alpha * v; });
  __syncthreads();
}

// dst(m x n) += src (global memory, no overlap)
__device__ inline void wg_add(int m, int n, const double* src, int lds, double* dst, int ldd) {
  const auto S = gmem(src);
  const auto D = gmem(dst);
  wg_each2(m, n, [&](int i, int j) { return make_double2(D[i + (int64_t)j * ldd], S[i + (int64_t)j * lds]); },
           [&](int i, int j, double2 v) { D[i + (int64_t)j * ldd] = v.x + v.y; });
}

__device__ inline void wg_fill(int m, int n, double* dst, int ldd, double v) {
  if (m > 0) {
    WG_FOR2(m, n, i, j) dst[i + (int64_t)j * ldd] = v;
  }
  __syncthreads();
}

// Pivot choice over the workgroup: every thread brings its best (|value|,
// row); all threads return the largest |value|, the smallest row on ties.
// Wave shuffles, then the four wave results through LDS (one barrier); the
// caller separates consecutive calls by at least one barrier.
__device__ inline void wg_argmax(double& v, int& idx) {
  __shared__ double wv[NT / 64];
  __shared__ int wi[NT / 64];
  for (int off = 32; off > 0; off >>= 1) {
    const double v2 = __shfl_xor(v, off, 64);
    const int i2 = __shfl_xor(idx, off, 64);
    if (v2 > v || (v2 == v && i2 < idx)) { v = v2; idx = i2; }
  }
  if ((threadIdx.x & 63) == 0) {
    wv[threadIdx.x >> 6] = v;
    wi[threadIdx.x >> 6] = idx;
  }
  __syncthreads();
  v = wv[0];
  idx = wi[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w)
    if (wv[w] > v || (wv[w] == v && wi[w] < idx)) { v = wv[w]; idx = wi[w]; }
}

// In-place LU with partial pivoting (row interchanges), A = P L U, L unit
// lower.  piv[j] = row swapped with row j at step j (0-based).  The pivot is
// the entry of largest magnitude, the first one on ties.  Returns (to every
// thread) the first step with an exactly zero pivot + 1, or 0.
__device__ inline int wg_getrf(int d, double* A, int lda, int32_t* piv) {
  __shared__ int s_info;
  if (threadIdx.x == 0) s_info = 0;
  __syncthreads();
  const int tid = threadIdx.x;
  for (int j = 0; j < d; ++j) {
    // start at the diagonal so that the pivot index stays in range even for a
    // column of NaNs (no comparison below succeeds then)
    double best = -1.0;
    int bi = j;
    for (int i = j + tid; i < d; i += NT) {
      const double v = fabs(A[i + (int64_t)j * lda]);
      if (v > best) { best = v; bi = i; }
    }
    wg_argmax(best, bi);
    const int p = bi;
    const double pv = best;
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
    if (rem > 0) {
      const double* colj = A + j + 1 + (int64_t)j * lda;
      WG_FOR2(rem, rem, ii, cc) {
        double* a = A + (j + 1 + ii) + (int64_t)(j + 1 + cc) * lda;
        *a -= colj[ii] * A[j + (int64_t)(j + 1 + cc) * lda];
      }
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
    const double* lj = LU + j + 1 + (int64_t)j * lda;
    WG_FOR2(rem, nc, ii, c) B[j + 1 + ii + (int64_t)c * ldb] -= lj[ii] * B[j + (int64_t)c * ldb];
    __syncthreads();
  }
  // backward: upper
  for (int j = d - 1; j >= 0; --j) {
    const double djj = LU[j + (int64_t)j * lda];
    for (int c = tid; c < nc; c += NT) B[j + (int64_t)c * ldb] /= djj;
    __syncthreads();
    if (j > 0) {
      const double* uj = LU + (int64_t)j * lda;
      WG_FOR2(j, nc, i, c) B[i + (int64_t)c * ldb] -= uj[i] * B[j + (int64_t)c * ldb];
    }
    __syncthreads();
  }
}

// Sum over the workgroup (every thread gets the total).
__device__ inline double wg_sum(double v) {
  __shared__ double s_part[NT / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) s_part[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) t += s_part[w];
  return t;
}

constexpr int TRD_MAXN = 2048;  // largest matrix the tridiagonal eigen-solver takes

// Number of eigenvalues of the tridiagonal (d, e) below x (Sturm sequence).
__device__ inline int sturm_count(int n, const double* d, const double* e, double x, double tiny) {
  double q = d[0] - x;
  int c = q < 0.0;
  for (int i = 1; i < n; ++i) {
    if (q == 0.0) q = tiny;
    q = d[i] - x - e[i - 1] * e[i - 1] / q;
    c += q < 0.0;
  }
  return c;
}

__device__ inline void wg_trd_eigenvalues(int n, const double* A, int lda, double* W, double* lam);

// Eigenvalues of a symmetric A (n x n, overwritten): Householder reduction to
// tridiagonal form (the reflectors v_k are left in A[k+1:, k], tau[k] = 1 if
// reflector k is applied), then bisection on Sturm counts.  W holds d, e and
// tau (3n); lam receives the eigenvalues in descending order.
// The rank-2 update of step k and the product S v of step k + 1 share one
// pass over the trailing matrix.
__device__ inline void wg_syev_values(int n, double* A, int lda, double* W, double* lam) {
  // sq takes the next product during the fused pass (sp holds the next
  // reflector then)
  __shared__ double sv[TRD_MAXN], sw[TRD_MAXN], sp[TRD_MAXN], sq[TRD_MAXN];  // 64 KiB
  double* d = W;
  double* e = W + n;
  double* tau = W + 2 * n;
  const int tid = threadIdx.x;
  // sp holds p = S v for the current step once `have_p` is set
  bool have_p = false;
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double* x = A + (k + 1) + (int64_t)k * lda;
    double part = 0.0;
    for (int i = 1 + tid; i < m; i += NT) part += x[i] * x[i];
    const double sig = wg_sum(part);
    const double x0 = x[0];
    if (sig == 0.0) {
      if (tid == 0) { e[k] = x0; tau[k] = 0.0; }
      have_p = false;
      __syncthreads();
      continue;
    }
    const double alpha = -copysign(sqrt(x0 * x0 + sig), x0);
    const double v0 = x0 - alpha;
    const double inv = 1.0 / sqrt(sig + v0 * v0);
    for (int i = tid; i < m; i += NT) sv[i] = (i == 0 ? v0 : x[i]) * inv;
    __syncthreads();
    if (tid == 0) { e[k] = alpha; tau[k] = 1.0; }
    for (int i = tid; i < m; i += NT) x[i] = sv[i];
    double* S = A + (k + 1) + (int64_t)(k + 1) * lda;
    if (!have_p) {
      // p = S v  (four independent partial sums pipeline the loads)
      for (int i = tid; i < m; i += NT) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int j = 0;
        for (; j + 3 < m; j += 4) {
          a0 += S[i + (int64_t)j * lda] * sv[j];
          a1 += S[i + (int64_t)(j + 1) * lda] * sv[j + 1];
          a2 += S[i + (int64_t)(j + 2) * lda] * sv[j + 2];
          a3 += S[i + (int64_t)(j + 3) * lda] * sv[j + 3];
        }
        for (; j < m; ++j) a0 += S[i + (int64_t)j * lda] * sv[j];
        sp[i] = (a0 + a1) + (a2 + a3);
      }
      __syncthreads();
    }
    double kp = 0.0;
    for (int i = tid; i < m; i += NT) kp += sp[i] * sv[i];
    const double K = wg_sum(kp);
    for (int i = tid; i < m; i += NT) sw[i] = sp[i] - K * sv[i];  // w = p - K v
    __syncthreads();
    // S -= 2 (v w^T + w v^T): first the leading column (the next x), then the
    // rest fused with the next product S' v'
    for (int i = tid; i < m; i += NT) S[i] -= 2.0 * (sv[i] * sw[0] + sw[i] * sv[0]);
    __syncthreads();
    const int m2 = m - 1;
    if (k + 3 < n && m2 > 0) {
      // next reflector from the updated column
      double* x2 = S + 1;  // A[k+2:, k+1]
      double part2 = 0.0;
      for (int i = 1 + tid; i < m2; i += NT) part2 += x2[i] * x2[i];
      const double sig2 = wg_sum(part2);
      const double y0 = x2[0];
      double inv2 = 0.0, v02 = 0.0;
      if (sig2 != 0.0) {
        const double alpha2 = -copysign(sqrt(y0 * y0 + sig2), y0);
        v02 = y0 - alpha2;
        inv2 = 1.0 / sqrt(sig2 + v02 * v02);
      }
      // sp <- v' (next reflector), kept aside in registers of the pass below
      double* vn = sp;  // reuse: p of this step is no longer needed
      for (int i = tid; i < m2; i += NT) vn[i] = sig2 != 0.0 ? (i == 0 ? v02 : x2[i]) * inv2 : 0.0;
      __syncthreads();
      // fused pass over S[1:, 1:]: update and accumulate S' v' into sq (rows
      // of this thread: i = tid + NT t, at most TRD_MAXN / NT of them)
      double* S2 = S + 1 + lda;
      for (int t = 0; t < TRD_MAXN / NT; ++t) {
        const int i = tid + NT * t;
        if (i >= m2) break;
        const double vi = sv[i + 1], wi = sw[i + 1];
        double a0 = 0.0, a1 = 0.0;
        int j = 0;
        // four columns per batch: their loads, then the updates (even
        // columns into a0, odd into a1, as below), then the stores
        for (; j + 3 < m2; j += 4) {
          double x[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) x[q] = gmem(S2)[i + (int64_t)(j + q) * lda];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            x[q] = x[q] - 2.0 * (vi * sw[j + q + 1] + wi * sv[j + q + 1]);
            if (q & 1) a1 += x[q] * vn[j + q];
            else a0 += x[q] * vn[j + q];
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) gmem(S2)[i + (int64_t)(j + q) * lda] = x[q];
        }
        for (; j + 1 < m2; j += 2) {
          double* c0 = S2 + i + (int64_t)j * lda;
          double* c1 = S2 + i + (int64_t)(j + 1) * lda;
          const double s0 = *c0 - 2.0 * (vi * sw[j + 1] + wi * sv[j + 1]);
          const double s1 = *c1 - 2.0 * (vi * sw[j + 2] + wi * sv[j + 2]);
          *c0 = s0;
          *c1 = s1;
          a0 += s0 * vn[j];
          a1 += s1 * vn[j + 1];
        }
        for (; j < m2; ++j) {
          double* c0 = S2 + i + (int64_t)j * lda;
          const double s0 = *c0 - 2.0 * (vi * sw[j + 1] + wi * sv[j + 1]);
          *c0 = s0;
          a0 += s0 * vn[j];
        }
        sq[i] = a0 + a1;
      }
      __syncthreads();
      // the next step recomputes its v from the same column; its p is S'' v'
      // (only when that reflector is non-trivial)
      if (sig2 != 0.0) {
        for (int i = tid; i < m2; i += NT) sp[i] = sq[i];
        have_p = true;
      } else {
        have_p = false;
      }
      __syncthreads();
    } else {
      WG_FOR2(m, m, ii, jj) if (jj > 0) S[ii + (int64_t)jj * lda] -= 2.0 * (sv[ii] * sw[jj] + sw[ii] * sv[jj]);
      have_p = false;
      __syncthreads();
    }
  }
  wg_trd_eigenvalues(n, A, lda, W, lam);
}

// After a Householder reduction that left e[0..n-3] and the reflectors in W /
// below the subdiagonal of A: the diagonal d, the last off-diagonal, then the
// eigenvalues by bisection on Sturm counts (one thread per eigenvalue),
// descending into lam.
__device__ inline void wg_trd_eigenvalues(int n, const double* A, int lda, double* W, double* lam) {
  __shared__ double s_lo, s_hi;
  double* d = W;
  double* e = W + n;
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += NT) d[i] = A[i + (int64_t)i * lda];
  if (tid == 0 && n >= 2) e[n - 2] = A[(n - 1) + (int64_t)(n - 2) * lda];
  __syncthreads();
  // Gershgorin interval
  if (tid == 0) {
    double lo = 0.0, hi = 0.0;
    for (int i = 0; i < n; ++i) {
      const double rad = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
      if (i == 0 || d[i] - rad < lo) lo = d[i] - rad;
      if (i == 0 || d[i] + rad > hi) hi = d[i] + rad;
    }
    s_lo = lo;
    s_hi = hi;
  }
  __syncthreads();
  const double lo = s_lo, hi = s_hi;
  const double nrm = fmax(fabs(lo), fabs(hi));
  const double tiny = 2.2e-16 * nrm + 1e-300;
  for (int j = tid; j < n; j += NT) {
    const int target = n - 1 - j;  // the j-th largest has n-1-j eigenvalues below it
    double a = lo, b = hi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (a + b);
      if (b - a <= 4.4e-16 * nrm || mid <= a || mid >= b) break;
      if (sturm_count(n, d, e, mid, tiny) > target) b = mid;
      else a = mid;
    }
    lam[j] = 0.5 * (a + b);
  }
  __syncthreads();
}

// Eigenvectors of the k largest eigenvalues (after wg_syev_values): inverse
// iteration on the tridiagonal (one thread per vector, pivoted LU of T - lam I),
// two passes of modified Gram-Schmidt, then the Householder back-transform
// (left to the caller when bt is false).
// X (n x k, ld ldx) receives the vectors; IW holds 5 n k doubles.
// The substitutions walk each vector in chunks of EV_CH rows: a chunk's loads
// are issued together before its serial recurrence, the results stored after.
constexpr int EV_CH = 8;
__device__ inline void wg_syev_vectors(int n, const double* A, int lda, const double* W, const double* lam, int k,
                                       double* X, int ldx, double* IW, bool bt = true) {
  __shared__ double s_c[NT];
  __shared__ double s_d[TRD_MAXN], s_e[TRD_MAXN];
  const auto tau = gmem(W + 2 * n);
  const int tid = threadIdx.x;
  if (k <= 0) return;
  if (n == 1) {
    if (tid == 0) X[0] = 1.0;
    __syncthreads();
    return;
  }
  for (int i = tid; i < n; i += NT) {
    s_d[i] = W[i];
    s_e[i] = W[n + i];
  }
  __syncthreads();
  const double* d = s_d;
  const double* e = s_e;
  const double nrm = fmax(fabs(lam[0]), fabs(lam[n - 1])) + 1e-300;
  const double tiny = 2.2e-16 * nrm;
  for (int j = tid; j < k; j += NT) {
    // interleaved per-thread arrays: element i of vector j at [i * k + j]
    const auto u0 = gmem(IW);
    const auto u1 = gmem(IW + (int64_t)n * k);
    const auto u2 = gmem(IW + 2 * (int64_t)n * k);
    const auto ll = gmem(IW + 3 * (int64_t)n * k);
    const auto pv = gmem(IW + 4 * (int64_t)n * k);
    const double mu = lam[j];
    // pivots below tiny in magnitude are stored as +-tiny
    auto clamp = [&](double u) { return fabs(u) < tiny ? ((u < 0.0) ? -tiny : tiny) : u; };
    double cd = d[0] - mu, cs = e[0];
    for (int i = 0; i + 1 < n; ++i) {
      const double ns = e[i], nd = d[i + 1] - mu, nsp = (i + 2 < n) ? e[i + 1] : 0.0;
      const int64_t o = (int64_t)i * k + j;
      if (fabs(cd) >= fabs(ns)) {
        if (cd == 0.0) cd = tiny;
        const double mlt = ns / cd;
        u0[o] = clamp(cd); u1[o] = cs; u2[o] = 0.0; ll[o] = mlt; pv[o] = 0.0;
        cd = nd - mlt * cs;
        cs = nsp;
      } else {
        const double mlt = cd / ns;
        u0[o] = clamp(ns); u1[o] = nd; u2[o] = nsp; ll[o] = mlt; pv[o] = 1.0;
        cd = cs - mlt * nd;
        cs = -mlt * nsp;
      }
    }
    {
      const int64_t o = (int64_t)(n - 1) * k + j;  // last row: only the diagonal is non-zero
      u0[o] = clamp(cd); u1[o] = 0.0; u2[o] = 0.0; ll[o] = 0.0; pv[o] = 0.0;
    }
    const auto x = gmem(X + (int64_t)j * ldx);
    // distinct pseudo-random start per vector: within a (near-)degenerate
    // cluster the iterates then span the cluster's eigenspace
    for (int i = 0; i < n; ++i) {
      uint32_t hsh = (uint32_t)i * 2654435761u ^ ((uint32_t)j * 2246822519u + 0x9E3779B9u);
      hsh = hsh * 747796405u + 2891336453u;
      hsh ^= hsh >> 16;
      hsh *= 2246822519u;
      hsh ^= hsh >> 13;
      x[i] = 0.25 + (double)(hsh >> 8) * (1.0 / 16777216.0);
    }
    for (int it = 0; it < 3; ++it) {
      // apply L (with the row interchanges), carrying b_i in a register
      double bi = x[0];
      for (int i0 = 0; i0 + 1 < n; i0 += EV_CH) {
        const int c = min(EV_CH, n - 1 - i0);
        double xb[EV_CH], pb[EV_CH], lb[EV_CH];
#pragma unroll
        for (int q = 0; q < EV_CH; ++q)
          if (q < c) {
            const int64_t o = (int64_t)(i0 + q) * k + j;
            xb[q] = x[i0 + 1 + q];
            pb[q] = pv[o];
            lb[q] = ll[o];
          }
#pragma unroll
        for (int q = 0; q < EV_CH; ++q)
          if (q < c) {
            double bn = xb[q];
            if (pb[q] != 0.0) { const double t = bi; bi = bn; bn = t; }
            xb[q] = bi;
            bi = bn - lb[q] * bi;
          }
#pragma unroll
        for (int q = 0; q < EV_CH; ++q)
          if (q < c) x[i0 + q] = xb[q];
      }
      x[n - 1] = bi;
      // back substitution with U (three diagonals)
      double x1 = 0.0, x2 = 0.0, ss = 0.0;
      for (int i1 = n; i1 > 0; i1 -= EV_CH) {
        const int c = min(EV_CH, i1);
        double xb[EV_CH], a0[EV_CH], a1[EV_CH], a2[EV_CH];
#pragma unroll
        for (int q = 0; q < EV_CH; ++q)
          if (q < c) {
            const int i = i1 - 1 - q;
            const int64_t o = (int64_t)i * k + j;
            xb[q] = x[i];
            a0[q] = u0[o];
            a1[q] = u1[o];
            a2[q] = u2[o];
          }
#pragma unroll
        for (int q = 0; q < EV_CH; ++q)
          if (q < c) {
            const double xi = (xb[q] - a1[q] * x1 - a2[q] * x2) / a0[q];
            xb[q] = xi;
            x2 = x1;
            x1 = xi;
            ss += xi * xi;
          }
#pragma unroll
        for (int q = 0; q < EV_CH; ++q)
          if (q < c) x[i1 - 1 - q] = xb[q];
      }
      const double sc = 1.0 / sqrt(ss);
      for (int i = 0; i < n; ++i) x[i] *= sc;
    }
  }
  __syncthreads();
  // Orthonormalisation, largest eigenvalue first: block classical Gram-Schmidt
  // with reorthogonalisation (blocks of 32 vectors projected against all
  // earlier ones by two in-workgroup GEMMs, twice), then Gram-Schmidt inside
  // the block.  IW (free after the inverse iteration) holds the coefficients.
  const int wave = tid >> 6, lane = tid & 63;
  const bool blocked = (int64_t)n * k * 5 >= (int64_t)32 * k + (int64_t)n * 32 + 32 * 32 + 64;
  for (int j0 = 0; j0 < k; j0 += 32) {
    const int jb = min(32, k - j0);
    if (j0 > 0 && blocked) {
      for (int pass = 0; pass < 2; ++pass) {
        wg_gemm(j0, jb, n, 1.0, X, ldx, true, X + (int64_t)j0 * ldx, ldx, false, 0.0, IW, j0);
        wg_gemm(n, jb, j0, -1.0, X, ldx, false, IW, j0, false, 1.0, X + (int64_t)j0 * ldx, ldx);
      }
    }
    const int jlo = blocked ? j0 : 0;
    for (int j = j0; j < j0 + jb; ++j) {
      double* xj = X + (int64_t)j * ldx;
      for (int pass = 0; pass < 2; ++pass) {
        for (int i0 = jlo; i0 < j; i0 += NT) {
          const int cnt = min(NT, j - i0);
          for (int i = i0 + wave; i < i0 + cnt; i += NT / 64) {
            const double* xi = X + (int64_t)i * ldx;
            double c = 0.0;
            for (int r = lane; r < n; r += 64) c += xi[r] * xj[r];
            for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
            if (lane == 0) s_c[i - i0] = c;
          }
          __syncthreads();
          for (int r = tid; r < n; r += NT) {
            double v = xj[r];
            for (int i = 0; i < cnt; ++i) v -= s_c[i] * X[r + (int64_t)(i0 + i) * ldx];
            xj[r] = v;
          }
          __syncthreads();
        }
      }
      double part = 0.0;
      for (int r = tid; r < n; r += NT) part += xj[r] * xj[r];
      const double nn = wg_sum(part);
      const double sc = 1.0 / sqrt(nn);
      for (int r = tid; r < n; r += NT) xj[r] *= sc;
      __syncthreads();
    }
  }
  if (!bt) return;
  // back-transform X <- H_0 H_1 ... H_{n-3} X, H_q = I - tq vq vq^T (tq = 2 or 0):
  // 32 reflectors at a time in compact WY form H_b0 ... H_b1-1 = I - V T V^T
  // (T upper triangular), applied as W = V^T X, W = T W, X -= V W.
  const int nref = n - 2;
  if (blocked && nref >= 32) {
    double* Vb = IW;                          // n x 32
    double* Tb = IW + (int64_t)n * 32;         // 32 x 32
    double* Wb = Tb + 32 * 32;                 // 32 x k
    for (int b1 = nref; b1 > 0; b1 -= 32) {
      const int b0 = max(0, b1 - 32), nb = b1 - b0;
      // V: column q - b0 holds v_q in rows q+1..n-1, zeros above
      WG_FOR2(n, nb, r, c) {
        const int q = b0 + c;
        Vb[r + (int64_t)c * n] = (r > q && tau[q] != 0.0) ? A[r + (int64_t)q * lda] : 0.0;
      }
      __syncthreads();
      // T: column c = -t_c T[0:c, 0:c] (V[:, 0:c]^T v_c), T[c][c] = t_c
      for (int c = 0; c < nb; ++c) {
        const double tc = tau[b0 + c] != 0.0 ? 2.0 : 0.0;
        for (int i = wave; i < c; i += NT / 64) {
          double g = 0.0;
          for (int r = lane; r < n; r += 64) g += Vb[r + (int64_t)i * n] * Vb[r + (int64_t)c * n];
          for (int off = 32; off > 0; off >>= 1) g += __shfl_xor(g, off, 64);
          if (lane == 0) s_c[i] = g;
        }
        __syncthreads();
        if (tid < c) {
          double acc = 0.0;
          for (int q = tid; q < c; ++q) acc += Tb[tid + q * 32] * s_c[q];
          Tb[tid + c * 32] = -tc * acc;
        }
        if (tid == c) Tb[c + c * 32] = tc;
        if (tid > c && tid < 32) Tb[tid + c * 32] = 0.0;
        __syncthreads();
      }
      wg_gemm(nb, k, n, 1.0, Vb, n, true, X, ldx, false, 0.0, Wb, 32);          // W = V^T X
      // W = T W (T upper triangular, in place by rows top-down)
      for (int j = tid; j < k; j += NT) {
        for (int i = 0; i < nb; ++i) {
          double acc = 0.0;
          for (int q = i; q < nb; ++q) acc += Tb[i + q * 32] * Wb[q + (int64_t)j * 32];
          Wb[i + (int64_t)j * 32] = acc;
        }
      }
      __syncthreads();
      wg_gemm(n, k, nb, -1.0, Vb, n, false, Wb, 32, false, 1.0, X, ldx);         // X -= V W
    }
  } else {
    for (int kk = n - 3; kk >= 0; --kk) {
      if (tau[kk] == 0.0) continue;
      const int m = n - kk - 1;
      const double* v = A + (kk + 1) + (int64_t)kk * lda;
      for (int j0 = 0; j0 < k; j0 += NT) {
        const int cnt = min(NT, k - j0);
        for (int j = j0 + wave; j < j0 + cnt; j += NT / 64) {
          const double* xj = X + (kk + 1) + (int64_t)j * ldx;
          double c = 0.0;
          for (int r = lane; r < m; r += 64) c += v[r] * xj[r];
          for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
          if (lane == 0) s_c[j - j0] = c;
        }
        __syncthreads();
        WG_FOR2(m, cnt, r, j) X[(kk + 1 + r) + (int64_t)(j0 + j) * ldx] -= 2.0 * s_c[j] * v[r];
        __syncthreads();
      }
    }
  }
}

// Symmetric eigen-decomposition by the cyclic Jacobi method with a parallel
// (round-robin) ordering: A (n x n, overwritten) = V diag(lam) V^T.  On return
// lam is sorted in descending order and V holds the matching eigenvectors.
// Vtmp (n x n) is workspace.
__device__ inline void wg_syev_jacobi(int n, double* A, int lda, double* V, int ldv, double* Vtmp, double* lam) {
  // one entry per rotation pair of a round: n <= 2 * JAC_MAXPAIR
  __shared__ double s_c[1024], s_s[1024];
  __shared__ int s_p[1024], s_q[1024];
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
