// Reduced energies of the analytic bias models on the device:
// u_kn = model_k(xi_n) for LINEAR (c_k + sum_j a_kj x_j) and HARMONIC
// (c_k + sum_j kappa_kj / 2 (x_j - x0_kj)^2) models, FP64, K x N with row
// stride N. One thread per sample keeps its coordinates in registers and
// walks the states; the coefficient reads are uniform across the wave and
// the writes of each state row are coalesced. Any common potential U(xi) is
// left out: it cancels between states in the MBAR equations (Sec. 2).
#include <cmath>

#include "bumbar.h"
#include "bumbar_impl.h"

namespace bumbar {

constexpr int kMT = 256;

template <int D>
__global__ void __launch_bounds__(kMT)
    model_energies_kernel(int K, int64_t N, int model, const double* __restrict__ coef,
                          const double* __restrict__ xi, double* __restrict__ u) {
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
    u[(int64_t)k * N + n] = v;
  }
}

hipError_t launch_model_energies(hipStream_t s, int K, int64_t N, int d, int model,
                                 const double* coef, const double* xi, double* u) {
  const dim3 grid((unsigned)((N + kMT - 1) / kMT));
  if (d == 1)
    hipLaunchKernelGGL(model_energies_kernel<1>, grid, dim3(kMT), 0, s, K, N, model, coef, xi, u);
  else
    hipLaunchKernelGGL(model_energies_kernel<2>, grid, dim3(kMT), 0, s, K, N, model, coef, xi, u);
  return hipGetLastError();
}

}  // namespace bumbar
