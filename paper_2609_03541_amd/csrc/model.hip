// Reduced energies of the analytic bias models on the device:
// u_kn = model_k(xi_n) for LINEAR (c_k + sum_j a_kj x_j) and HARMONIC
// (c_k + sum_j kappa_kj / 2 (x_j - x0_kj)^2) models, FP64, K x N with row
// stride N. One thread per sample keeps its coordinates in registers and
// walks the states; the coefficient reads are uniform across the wave and
// the writes of each state row are coalesced. Any common potential U(xi) is
// left out: it cancels between states in the MBAR equations (Sec. 2).
#include <algorithm>
#include <cmath>

#include "bumbar.h"
#include "bumbar_impl.h"

namespace bumbar {

constexpr int kMT = 256;

template <int D, typename TO>
__global__ void __launch_bounds__(kMT)
    model_energies_kernel(int K, int64_t N, int model, const double* __restrict__ coef,
                          const double* __restrict__ xi, TO* __restrict__ u) {
  const int64_t n = (int64_t)blockIdx.x * kMT + threadIdx.x;
  if (n >= N) return;
  double x[D];
#pragma unroll
  for (int j = 0; j < D; ++j) x[j] = xi[n * D + j];
  for (int k = 0; k < K; ++k) {
    const double* ck = coef + (int64_t)k * (1 + 2 * D);
    double v = ck[0];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (model == BUMBAR_MODEL_LINEAR) {
        v += ck[1 + j] * x[j];
      } else {
        const double dx = x[j] - ck[2 + 2 * j];
        v += 0.5 * ck[1 + 2 * j] * dx * dx;
      }
    }
    u[(int64_t)k * N + n] = (TO)v;
  }
}

hipError_t launch_model_energies(hipStream_t s, int K, int64_t N, int d, int model,
                                 const double* coef, const double* xi, void* u, bool f32) {
  const dim3 grid((unsigned)((N + kMT - 1) / kMT));
  if (f32) {
    // FP64 model values rounded once to the FP32 storage type
    float* uf = static_cast<float*>(u);
    if (d == 1)
      hipLaunchKernelGGL((model_energies_kernel<1, float>), grid, dim3(kMT), 0, s, K, N, model,
                         coef, xi, uf);
    else
      hipLaunchKernelGGL((model_energies_kernel<2, float>), grid, dim3(kMT), 0, s, K, N, model,
                         coef, xi, uf);
  } else {
    double* ud = static_cast<double*>(u);
    if (d == 1)
      hipLaunchKernelGGL((model_energies_kernel<1, double>), grid, dim3(kMT), 0, s, K, N, model,
                         coef, xi, ud);
    else
      hipLaunchKernelGGL((model_energies_kernel<2, double>), grid, dim3(kMT), 0, s, K, N, model,
                         coef, xi, ud);
  }
  return hipGetLastError();
}

__global__ void __launch_bounds__(kMT)
    widen_f32_kernel(const float* __restrict__ src, int64_t n, double* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * kMT;
  for (int64_t i = (int64_t)blockIdx.x * kMT + threadIdx.x; i < n; i += stride)
    dst[i] = (double)src[i];
}

hipError_t launch_widen_f32(hipStream_t s, const float* src, int64_t n, double* dst) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + kMT - 1) / kMT, 8192);
  hipLaunchKernelGGL(widen_f32_kernel, dim3((unsigned)blocks), dim3(kMT), 0, s, src, n, dst);
  return hipGetLastError();
}

}  // namespace bumbar
