// Rank-prediction network: device forward pass used inside the factorisation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ifmm {

// y[i] = network(theta, X[i, :]) for m samples of F features (row-major), on
// stream s; work must hold mlp_work_floats(m) floats.  Returns 0 or -3.
int mlp_forward_dev(const float* theta, int F, const float* X, int64_t m, float* y, float* work, hipStream_t s);
int64_t mlp_work_floats(int64_t m);

}  // namespace ifmm
