// Rank-prediction network on the device: forward, pinball-loss backward and
// Adam, FP32 parameters and activations, FP64 accumulation of the parameter
// gradients over the samples (fixed order, so training is deterministic).
//
// Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3,
// 64 units per hidden layer.  Flat parameter order: W1 (64 x F, row-major),
// b1 (64), W2 (64 x 64, row-major), b2 (64), w3 (64), b3 (1).  Loss: mean
// pinball loss at quantile tau of u = target - y, subgradient -tau at u = 0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/ifmm.h"
#include "mlp.hpp"

namespace ifmm {

constexpr int MH = 64;
constexpr int MNT = 256;

static inline int64_t mlp_np(int F) { return (int64_t)MH * F + MH + MH * MH + MH + MH + 1; }

__global__ void __launch_bounds__(MNT) k_mlp_layer1(const float* th, int F, const float* X, int64_t m, float* Z1, float* H1) {
  const int64_t e = (int64_t)blockIdx.x * MNT + threadIdx.x;
  if (e >= m * MH) return;
  const int64_t i = e / MH;
  const int j = (int)(e - i * MH);
  const float* W1 = th;
  const float* b1 = th + (int64_t)MH * F;
  float z = b1[j];
  for (int f = 0; f < F; ++f) z = fmaf(W1[j * F + f], X[i * F + f], z);
  Z1[e] = z;
  H1[e] = z > 0.f ? z : 0.f;
}

__global__ void __launch_bounds__(MNT) k_mlp_layer2(const float* th, int F, const float* H1, int64_t m, float* Z2, float* H2) {
  const int64_t e = (int64_t)blockIdx.x * MNT + threadIdx.x;
  if (e >= m * MH) return;
  const int64_t i = e / MH;
  const int j = (int)(e - i * MH);
  const float* W2 = th + (int64_t)MH * F + MH;
  const float* b2 = W2 + MH * MH;
  float z = b2[j];
  for (int k = 0; k < MH; ++k) z = fmaf(W2[j * MH + k], H1[i * MH + k], z);
  Z2[e] = z;
  H2[e] = z > 0.f ? z : 0.f;
}

__global__ void __launch_bounds__(MNT) k_mlp_out(const float* th, int F, const float* H2, int64_t m, float* Y) {
  const int64_t i = (int64_t)blockIdx.x * MNT + threadIdx.x;
  if (i >= m) return;
  const float* w3 = th + (int64_t)MH * F + MH + MH * MH + MH;
  float y = w3[MH];
  for (int j = 0; j < MH; ++j) y = fmaf(w3[j], H2[i * MH + j], y);
  Y[i] = y;
}

// dL/dy (sample i) and the per-sample loss
__global__ void __launch_bounds__(MNT) k_mlp_dy(const float* Y, const float* T, int64_t m, float tau, float* DY, float* Lterm) {
  const int64_t i = (int64_t)blockIdx.x * MNT + threadIdx.x;
  if (i >= m) return;
  const float u = T[i] - Y[i];
  DY[i] = (u >= 0.f ? -tau : 1.f - tau) / (float)m;
  Lterm[i] = u >= 0.f ? tau * u : (tau - 1.f) * u;
}

__global__ void __launch_bounds__(MNT) k_mlp_dz2(const float* th, int F, const float* DY, const float* Z2, int64_t m, float* DZ2) {
  const int64_t e = (int64_t)blockIdx.x * MNT + threadIdx.x;
  if (e >= m * MH) return;
  const int64_t i = e / MH;
  const int j = (int)(e - i * MH);
  const float* w3 = th + (int64_t)MH * F + MH + MH * MH + MH;
  DZ2[e] = Z2[e] > 0.f ? DY[i] * w3[j] : 0.f;
}

__global__ void __launch_bounds__(MNT) k_mlp_dz1(const float* th, int F, const float* DZ2, const float* Z1, int64_t m, float* DZ1) {
  const int64_t e = (int64_t)blockIdx.x * MNT + threadIdx.x;
  if (e >= m * MH) return;
  const int64_t i = e / MH;
  const int k = (int)(e - i * MH);
  const float* W2 = th + (int64_t)MH * F + MH;
  float s = 0.f;
  for (int j = 0; j < MH; ++j) s = fmaf(DZ2[i * MH + j], W2[j * MH + k], s);
  DZ1[e] = Z1[e] > 0.f ? s : 0.f;
}

// one thread per parameter: sum over the samples in FP64
__global__ void __launch_bounds__(MNT) k_mlp_pgrad(int F, const float* X, const float* H1, const float* H2, const float* DY, const float* DZ1,
                            const float* DZ2, int64_t m, float* G) {
  const int64_t p = (int64_t)blockIdx.x * MNT + threadIdx.x;
  const int64_t o1 = (int64_t)MH * F, o2 = o1 + MH, o3 = o2 + MH * MH, o4 = o3 + MH, o5 = o4 + MH, o6 = o5 + 1;
  if (p >= o6) return;
  double s = 0.0;
  if (p < o1) {
    const int j = (int)(p / F), f = (int)(p % F);
    for (int64_t i = 0; i < m; ++i) s += (double)DZ1[i * MH + j] * X[i * F + f];
  } else if (p < o2) {
    const int j = (int)(p - o1);
    for (int64_t i = 0; i < m; ++i) s += DZ1[i * MH + j];
  } else if (p < o3) {
    const int j = (int)((p - o2) / MH), k = (int)((p - o2) % MH);
    for (int64_t i = 0; i < m; ++i) s += (double)DZ2[i * MH + j] * H1[i * MH + k];
  } else if (p < o4) {
    const int j = (int)(p - o3);
    for (int64_t i = 0; i < m; ++i) s += DZ2[i * MH + j];
  } else if (p < o5) {
    const int j = (int)(p - o4);
    for (int64_t i = 0; i < m; ++i) s += (double)DY[i] * H2[i * MH + j];
  } else {
    for (int64_t i = 0; i < m; ++i) s += DY[i];
  }
  G[p] = (float)s;
}

__global__ void __launch_bounds__(MNT) k_mlp_adam(float* th, const float* g, float* m1, float* m2, int64_t n, float lr, float c1, float c2) {
  const int64_t p = (int64_t)blockIdx.x * MNT + threadIdx.x;
  if (p >= n) return;
  const float a = 0.9f * m1[p] + 0.1f * g[p];
  const float b = 0.999f * m2[p] + 0.001f * g[p] * g[p];
  m1[p] = a;
  m2[p] = b;
  th[p] -= lr * (a / c1) / (sqrtf(b / c2) + 1e-8f);
}

__global__ void __launch_bounds__(MNT) k_mlp_sum(const float* v, int64_t m, double* out) {
  __shared__ double red[MNT];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += MNT) s += v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = MNT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

static unsigned blocks(int64_t n) { return (unsigned)((n + MNT - 1) / MNT); }

int mlp_forward_dev(const float* th, int F, const float* X, int64_t m, float* Y, float* work, hipStream_t s) {
  if (m <= 0) return 0;
  float* Z1 = work;
  float* H1 = Z1 + m * MH;
  float* Z2 = H1 + m * MH;
  float* H2 = Z2 + m * MH;
  hipLaunchKernelGGL(k_mlp_layer1, dim3(blocks(m * MH)), dim3(MNT), 0, s, th, F, X, m, Z1, H1);
  hipLaunchKernelGGL(k_mlp_layer2, dim3(blocks(m * MH)), dim3(MNT), 0, s, th, F, H1, m, Z2, H2);
  hipLaunchKernelGGL(k_mlp_out, dim3(blocks(m)), dim3(MNT), 0, s, th, F, H2, m, Y);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int64_t mlp_work_floats(int64_t m) { return 4 * m * MH + 8; }

// loss and gradient on the device (buffers: work of 7 m MH + 4 m floats)
static void mlp_grad_dev(const float* th, int F, const float* X, const float* T, int64_t m, float tau, float* G,
                         float* work, double* dloss, hipStream_t s) {
  float* Z1 = work;
  float* H1 = Z1 + m * MH;
  float* Z2 = H1 + m * MH;
  float* H2 = Z2 + m * MH;
  float* DZ2 = H2 + m * MH;
  float* DZ1 = DZ2 + m * MH;
  float* Y = DZ1 + m * MH;
  float* DY = Y + m;
  float* LT = DY + m;
  hipLaunchKernelGGL(k_mlp_layer1, dim3(blocks(m * MH)), dim3(MNT), 0, s, th, F, X, m, Z1, H1);
  hipLaunchKernelGGL(k_mlp_layer2, dim3(blocks(m * MH)), dim3(MNT), 0, s, th, F, H1, m, Z2, H2);
  hipLaunchKernelGGL(k_mlp_out, dim3(blocks(m)), dim3(MNT), 0, s, th, F, H2, m, Y);
  hipLaunchKernelGGL(k_mlp_dy, dim3(blocks(m)), dim3(MNT), 0, s, Y, T, m, tau, DY, LT);
  hipLaunchKernelGGL(k_mlp_dz2, dim3(blocks(m * MH)), dim3(MNT), 0, s, th, F, DY, Z2, m, DZ2);
  hipLaunchKernelGGL(k_mlp_dz1, dim3(blocks(m * MH)), dim3(MNT), 0, s, th, F, DZ2, Z1, m, DZ1);
  hipLaunchKernelGGL(k_mlp_pgrad, dim3(blocks(mlp_np(F))), dim3(MNT), 0, s, F, X, H1, H2, DY, DZ1, DZ2, m, G);
  if (dloss) hipLaunchKernelGGL(k_mlp_sum, dim3(1), dim3(MNT), 0, s, LT, m, dloss);
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace ifmm

using namespace ifmm;

extern "C" {

int64_t ifmm_rank_model_params(int32_t nfeat) { return nfeat < 1 ? -1 : mlp_np(nfeat); }

ifmm_status ifmm_rank_model_eval(const float* theta, int32_t F, const float* X, int64_t m, float* y) {
  if (!theta || !X || !y || F < 1 || m < 1) return IFMM_EINVAL;
  const int64_t np = mlp_np(F);
  DevBuf b;
  const int64_t tot = np + m * F + m + mlp_work_floats(m);
  if (hipMalloc(&b.p, tot * 4) != hipSuccess) return IFMM_ENOMEM;
  float* dth = (float*)b.p;
  float* dX = dth + np;
  float* dY = dX + m * F;
  float* dW = dY + m;
  if (hipMemcpy(dth, theta, np * 4, hipMemcpyHostToDevice) != hipSuccess) return IFMM_EDEVICE;
  if (hipMemcpy(dX, X, m * F * 4, hipMemcpyHostToDevice) != hipSuccess) return IFMM_EDEVICE;
  if (mlp_forward_dev(dth, F, dX, m, dY, dW, nullptr)) return IFMM_EDEVICE;
  if (hipMemcpy(y, dY, m * 4, hipMemcpyDeviceToHost) != hipSuccess) return IFMM_EDEVICE;
  return IFMM_OK;
}

ifmm_status ifmm_rank_model_grad(const float* theta, int32_t F, const float* X, const float* t, int64_t m, float tau,
                         double* loss, float* grad) {
  if (!theta || !X || !t || !grad || F < 1 || m < 1) return IFMM_EINVAL;
  const int64_t np = mlp_np(F);
  DevBuf b;
  const int64_t tot = 2 * np + m * F + m + 6 * m * MH + 3 * m + 16;
  if (hipMalloc(&b.p, tot * 4) != hipSuccess) return IFMM_ENOMEM;
  float* dth = (float*)b.p;
  float* dG = dth + np;
  float* dX = dG + np;
  float* dT = dX + m * F;
  float* dW = dT + m;
  double* dL = nullptr;
  if (hipMalloc((void**)&dL, 8) != hipSuccess) return IFMM_ENOMEM;
  DevBuf bl;
  bl.p = dL;
  if (hipMemcpy(dth, theta, np * 4, hipMemcpyHostToDevice) != hipSuccess) return IFMM_EDEVICE;
  if (hipMemcpy(dX, X, m * F * 4, hipMemcpyHostToDevice) != hipSuccess) return IFMM_EDEVICE;
  if (hipMemcpy(dT, t, m * 4, hipMemcpyHostToDevice) != hipSuccess) return IFMM_EDEVICE;
  mlp_grad_dev(dth, F, dX, dT, m, tau, dG, dW, dL, nullptr);
  if (hipMemcpy(grad, dG, np * 4, hipMemcpyDeviceToHost) != hipSuccess) return IFMM_EDEVICE;
  double Ls = 0.0;
  if (hipMemcpy(&Ls, dL, 8, hipMemcpyDeviceToHost) != hipSuccess) return IFMM_EDEVICE;
  if (loss) *loss = Ls / (double)m;
  return IFMM_OK;
}

// Full-batch Adam on the device for `steps` steps from theta (updated in place);
// loss_hist[k] = loss before step k + 1 (may be NULL).
ifmm_status ifmm_rank_model_train(const float* X, const float* t, int64_t m, int32_t F, int32_t steps, float lr, float tau,
                          float* theta, double* loss_hist) {
  if (!X || !t || !theta || F < 1 || m < 1 || steps < 0 || !(lr > 0.f) || !(tau > 0.f && tau < 1.f)) return IFMM_EINVAL;
  const int64_t np = mlp_np(F);
  DevBuf b, bl;
  const int64_t tot = 4 * np + m * F + m + 6 * m * MH + 3 * m + 16;
  if (hipMalloc(&b.p, tot * 4) != hipSuccess) return IFMM_ENOMEM;
  if (hipMalloc(&bl.p, std::max<int64_t>(steps, 1) * 8) != hipSuccess) return IFMM_ENOMEM;
  float* dth = (float*)b.p;
  float* dG = dth + np;
  float* dm1 = dG + np;
  float* dm2 = dm1 + np;
  float* dX = dm2 + np;
  float* dT = dX + m * F;
  float* dW = dT + m;
  double* dL = (double*)bl.p;
  if (hipMemcpy(dth, theta, np * 4, hipMemcpyHostToDevice) != hipSuccess) return IFMM_EDEVICE;
  if (hipMemset(dm1, 0, 2 * np * 4) != hipSuccess) return IFMM_EDEVICE;
  if (hipMemcpy(dX, X, m * F * 4, hipMemcpyHostToDevice) != hipSuccess) return IFMM_EDEVICE;
  if (hipMemcpy(dT, t, m * 4, hipMemcpyHostToDevice) != hipSuccess) return IFMM_EDEVICE;
  for (int k = 1; k <= steps; ++k) {
    mlp_grad_dev(dth, F, dX, dT, m, tau, dG, dW, dL + (k - 1), nullptr);
    const float c1 = 1.f - std::pow(0.9f, (float)k), c2 = 1.f - std::pow(0.999f, (float)k);
    hipLaunchKernelGGL(k_mlp_adam, dim3(blocks(np)), dim3(MNT), 0, nullptr, dth, dG, dm1, dm2, np, lr, c1, c2);
  }
  if (hipDeviceSynchronize() != hipSuccess) return IFMM_EDEVICE;
  if (hipMemcpy(theta, dth, np * 4, hipMemcpyDeviceToHost) != hipSuccess) return IFMM_EDEVICE;
  if (loss_hist && steps > 0) {
    std::vector<double> h(steps);
    if (hipMemcpy(h.data(), dL, steps * 8, hipMemcpyDeviceToHost) != hipSuccess) return IFMM_EDEVICE;
    for (int k = 0; k < steps; ++k) loss_hist[k] = h[k] / (double)m;
  }
  return IFMM_OK;
}

}  // extern "C"
