// Newton direction of the MBAR objective on the reduced system.
//
// H annihilates the constant vector over sampled states (the gauge freedom of
// f), so the first sampled state and the unsampled states are dropped and the
// remaining m x m system H_RR d_R = -g_R (g = S - N) is solved in FP64 by an
// L D L^T factorisation (unit lower L, diagonal D): at step j every trailing
// element A_ik (j < k <= i) loses A_ij A_kj / A_jj, which needs one barrier
// per column and no square roots; the forward and backward substitutions take
// one barrier per column each. One workgroup runs the whole solve; the matrix
// sits in LDS when it fits (m <= 136) and in the workspace otherwise. A pivot
// that is not positive means the reduced Hessian is not positive definite
// (disconnected overlap): ok = 0 is reported and the host takes a
// self-consistent step instead.
#include <cmath>

#include "bumbar_impl.h"

namespace bumbar {

constexpr int kLT = 256;  // 16 x 16 threads
constexpr int kLdsMaxM = 136;  // 136^2 + 3 * 136 doubles < 150 KB of LDS

template <bool LDSMAT>
__global__ void __launch_bounds__(kLT)
    newton_direction_kernel(int K, const int64_t* __restrict__ Nk, const double* __restrict__ H,
                            const double* __restrict__ S, double* __restrict__ Aglob,
                            int* __restrict__ idx, double* __restrict__ d, int* __restrict__ ok) {
  extern __shared__ double dyn[];
  __shared__ int m_sh;
  __shared__ int bad_sh;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  if (tid == 0) {
    int m = 0, r = -1;
    for (int k = 0; k < K; ++k) {
      if (Nk[k] <= 0) continue;
      if (r < 0) {
        r = k;
        continue;
      }
      idx[m++] = k;
    }
    m_sh = m;
    bad_sh = 0;
  }
  for (int k = tid; k < K; k += kLT) d[k] = 0.0;
  __syncthreads();
  const int m = m_sh;
  double* A = LDSMAT ? dyn : Aglob;
  double* b = A + (int64_t)m * m;  // right-hand side, then two work vectors
  for (int64_t e = tid; e < (int64_t)m * m; e += kLT) {
    const int a = (int)(e / m), c = (int)(e % m);
    A[e] = H[(int64_t)idx[a] * K + idx[c]];
  }
  for (int a = tid; a < m; a += kLT) b[a] = -(S[idx[a]] - (double)Nk[idx[a]]);
  __syncthreads();
  // L D L^T: after step j, column j below the diagonal holds L_ij * D_j and
  // A_jj holds D_j.
  for (int j = 0; j < m; ++j) {
    const double p = A[(int64_t)j * m + j];
    if (!(p > 0.0)) {
      if (tid == 0) bad_sh = 1;
      break;  // uniform: every thread read the same pivot
    }
    const double rp = 1.0 / p;
    for (int i = j + 1 + ty; i < m; i += 16) {
      const double aij = A[(int64_t)i * m + j] * rp;
      for (int k = j + 1 + tx; k <= i; k += 16) A[(int64_t)i * m + k] -= aij * A[(int64_t)k * m + j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad_sh) {
    if (tid == 0) *ok = 0;
    return;
  }
  // forward: L y = b with L_ij = A_ij / A_jj (column oriented)
  for (int j = 0; j < m; ++j) {
    const double yj = b[j];
    const double rj = yj / A[(int64_t)j * m + j];
    for (int i = j + 1 + tid; i < m; i += kLT) b[i] -= A[(int64_t)i * m + j] * rj;
    __syncthreads();
  }
  // z = D^{-1} y
  for (int i = tid; i < m; i += kLT) b[i] /= A[(int64_t)i * m + i];
  // backward: L^T x = z, x_j = z_j - t_j / D_j with t_j = sum_{i > j} A_ij x_i
  double* t = b + m;
  double* x = t + m;
  for (int i = tid; i < m; i += kLT) t[i] = 0.0;
  __syncthreads();
  for (int j = m - 1; j >= 0; --j) {
    const double xj = b[j] - t[j] / A[(int64_t)j * m + j];
    if (tid == 0) x[j] = xj;
    for (int i = tid; i < j; i += kLT) t[i] += A[(int64_t)j * m + i] * xj;
    __syncthreads();
  }
  for (int a = tid; a < m; a += kLT) d[idx[a]] = x[a];
  if (tid == 0) *ok = 1;
}

hipError_t launch_newton_direction(hipStream_t s, int K, const int64_t* Nk, const double* H,
                                   const double* S, double* A, int* idx, double* d, int* ok) {
  // K - 1 bounds the reduced size m from above
  const int mmax = K - 1;
  if (mmax <= kLdsMaxM) {
    const size_t lds = sizeof(double) * ((size_t)mmax * mmax + 3 * mmax + 1);
    // raise the dynamic LDS limit once to the largest size this kernel uses
    static const bool attr = [] {
      const size_t mx = sizeof(double) * ((size_t)kLdsMaxM * kLdsMaxM + 3 * kLdsMaxM + 1);
      if (hipFuncSetAttribute(reinterpret_cast<const void*>(&newton_direction_kernel<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)mx) != hipSuccess)
        (void)hipGetLastError();  // clear; a launch that still fails reports it
      return true;
    }();
    (void)attr;
    hipLaunchKernelGGL(newton_direction_kernel<true>, dim3(1), dim3(kLT), lds, s, K, Nk, H, S, A,
                       idx, d, ok);
  } else {
    hipLaunchKernelGGL(newton_direction_kernel<false>, dim3(1), dim3(kLT), 0, s, K, Nk, H, S, A,
                       idx, d, ok);
  }
  return hipGetLastError();
}

}  // namespace bumbar
