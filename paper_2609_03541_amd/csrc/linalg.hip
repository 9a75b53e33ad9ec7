// Newton direction of the MBAR objective on the reduced system.
//
// H annihilates the constant vector over sampled states (the gauge freedom of
// f), so the first sampled state and the unsampled states are dropped and the
// remaining m x m system H_RR d_R = -g_R (g = S - N) is solved by a dense
// Cholesky factorisation in FP64. One workgroup of 1024 threads runs the
// whole factorisation (right-looking, column by column) and the two
// triangular solves; the matrix lives in the workspace (L2/MALL resident for
// the K of these workloads). If a pivot is not positive the system is not
// positive definite (disconnected overlap) and ok = 0 is reported; the host
// then takes a self-consistent step instead.
#include <cmath>

#include "bumbar_impl.h"

namespace bumbar {

constexpr int kLT = 1024;

__global__ void __launch_bounds__(kLT)
    newton_direction_kernel(int K, const int64_t* __restrict__ Nk, const double* __restrict__ H,
                            const double* __restrict__ S, double* __restrict__ A,
                            int* __restrict__ idx, double* __restrict__ d, int* __restrict__ ok) {
  __shared__ int m_sh;
  __shared__ int bad_sh;
  __shared__ double piv_sh;
  const int tid = threadIdx.x;
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
  double* b = A + (int64_t)m * m;  // right-hand side after the matrix
  for (int64_t e = tid; e < (int64_t)m * m; e += kLT) {
    const int a = (int)(e / m), c = (int)(e % m);
    A[e] = H[(int64_t)idx[a] * K + idx[c]];
  }
  for (int a = tid; a < m; a += kLT) b[a] = -(S[idx[a]] - (double)Nk[idx[a]]);
  __syncthreads();
  // Cholesky A = L L^T (lower triangle in place)
  for (int j = 0; j < m; ++j) {
    if (tid == 0) {
      const double p = A[(int64_t)j * m + j];
      if (!(p > 0.0) || p != p) bad_sh = 1;
      piv_sh = sqrt(p);
      A[(int64_t)j * m + j] = piv_sh;
    }
    __syncthreads();
    if (bad_sh) break;
    const double l = piv_sh;
    for (int i = j + 1 + tid; i < m; i += kLT) A[(int64_t)i * m + j] /= l;
    __syncthreads();
    // trailing update of the lower triangle: A_ik -= L_ij L_kj, j < k <= i
    const int64_t rem = m - j - 1;
    const int64_t cnt = rem * (rem + 1) / 2;
    for (int64_t e = tid; e < cnt; e += kLT) {
      // e -> (i, k) in the lower triangle of the trailing block, row-major
      int64_t ii = (int64_t)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
      while (ii * (ii + 1) / 2 > e) --ii;
      while ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
      const int64_t kk = e - ii * (ii + 1) / 2;
      const int64_t i = j + 1 + ii, k = j + 1 + kk;
      A[i * m + k] -= A[i * m + j] * A[k * m + j];
    }
    __syncthreads();
  }
  if (bad_sh) {
    if (tid == 0) *ok = 0;
    return;
  }
  // forward substitution L y = b (column oriented)
  for (int j = 0; j < m; ++j) {
    if (tid == 0) b[j] /= A[(int64_t)j * m + j];
    __syncthreads();
    const double bj = b[j];
    for (int i = j + 1 + tid; i < m; i += kLT) b[i] -= A[(int64_t)i * m + j] * bj;
    __syncthreads();
  }
  // back substitution L^T x = y
  for (int j = m - 1; j >= 0; --j) {
    if (tid == 0) b[j] /= A[(int64_t)j * m + j];
    __syncthreads();
    const double bj = b[j];
    for (int i = tid; i < j; i += kLT) b[i] -= A[(int64_t)j * m + i] * bj;
    __syncthreads();
  }
  for (int a = tid; a < m; a += kLT) d[idx[a]] = b[a];
  if (tid == 0) *ok = 1;
}

hipError_t launch_newton_direction(hipStream_t s, int K, const int64_t* Nk, const double* H,
                                   const double* S, double* A, int* idx, double* d, int* ok) {
  hipLaunchKernelGGL(newton_direction_kernel, dim3(1), dim3(kLT), 0, s, K, Nk, H, S, A, idx, d,
                     ok);
  return hipGetLastError();
}

}  // namespace bumbar
