// Chebyshev interpolation helpers of the black-box FMM (device, inline).
#pragma once

#include <hip/hip_runtime.h>

namespace ifmm {

// ------------------------------------------------------------------ Chebyshev
// Interpolation weight S_n(xb_m, y) = 1/n + (2/n) sum_{k=1}^{n-1} T_k(xb_m) T_k(y),
// xb_m = cos((2m + 1) pi / (2n)), m = 0..n-1.
__device__ inline double cheb_S(int nc, int m, double y) {
  const double xb = cos((2.0 * m + 1.0) * M_PI / (2.0 * nc));
  double s = 1.0 / nc;
  double tx0 = 1.0, tx1 = xb, ty0 = 1.0, ty1 = y;
  for (int k = 1; k < nc; ++k) {
    s += (2.0 / nc) * tx1 * ty1;
    const double tx2 = 2.0 * xb * tx1 - tx0, ty2 = 2.0 * y * ty1 - ty0;
    tx0 = tx1; tx1 = tx2; ty0 = ty1; ty1 = ty2;
  }
  return s;
}

__device__ inline double cheb_node(int nc, int m) { return cos((2.0 * m + 1.0) * M_PI / (2.0 * nc)); }

}  // namespace ifmm
