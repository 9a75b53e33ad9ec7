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
#include <algorithm>
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

int newton_lds_max_m() { return kLdsMaxM; }

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

// ---------------------------------------------------------------------------
// Reduced systems larger than the LDS kernel holds (m > 136): a blocked
// right-looking Cholesky factorisation A = L L^T in place (lower triangle,
// 64 x 64 blocks) followed by blocked forward and backward substitution. Per
// block column p: the diagonal block is factored by one workgroup in LDS,
// the blocks below it are solved against L_pp^T (one workgroup per block
// row), and every trailing block (i, j), p < j <= i, loses L_ip L_jp^T (one
// workgroup per block, 4 x 4 outputs per thread). A pivot that is not
// positive clears *ok, as in the LDS kernel.
namespace bumbar {

constexpr int CB = 64;       // Cholesky block edge
constexpr int CBP = CB + 1;  // padded LDS row

// A (m x m, row-major) = H[idx, idx], b = -(S - N)[idx], d = 0 elsewhere.
__global__ void reduced_gather_kernel(int K, int m, const int* __restrict__ idx,
                                      const double* __restrict__ H, const double* __restrict__ S,
                                      const int64_t* __restrict__ Nk, double* __restrict__ A,
                                      double* __restrict__ b, double* __restrict__ d) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < (int64_t)m * m) {
    const int r = (int)(e / m), c = (int)(e % m);
    A[e] = H[(int64_t)idx[r] * K + idx[c]];
  }
  if (e < m) b[e] = -(S[idx[e]] - (double)Nk[idx[e]]);
  if (e < K) d[e] = 0.0;
}

__global__ void __launch_bounds__(256)
    chol_diag_kernel(int m, int p, double* __restrict__ A, int* __restrict__ ok) {
  __shared__ double T[CB][CBP];
  __shared__ int bad;
  const int r0 = p * CB;
  const int nb = min(CB, m - r0);
  for (int e = threadIdx.x; e < CB * CB; e += 256) {
    const int r = e / CB, c = e % CB;
    T[r][c] = (r < nb && c < nb) ? A[(int64_t)(r0 + r) * m + r0 + c] : (r == c ? 1.0 : 0.0);
  }
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < CB; ++j) {
    const double piv = T[j][j];
    if (!(piv > 0.0)) {
      if (threadIdx.x == 0) bad = 1;
      break;  // uniform: every thread read the same pivot
    }
    const double l = sqrt(piv);
    __syncthreads();
    // column j below the diagonal, then the trailing lower triangle
    for (int i = j + 1 + threadIdx.x; i < CB; i += 256) T[i][j] /= l;
    if (threadIdx.x == 0) T[j][j] = l;
    __syncthreads();
    for (int e = threadIdx.x; e < (CB - j - 1) * (CB - j - 1); e += 256) {
      const int i = j + 1 + e / (CB - j - 1), k = j + 1 + e % (CB - j - 1);
      if (k <= i) T[i][k] -= T[i][j] * T[k][j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) {
    if (threadIdx.x == 0) *ok = 0;
    return;
  }
  for (int e = threadIdx.x; e < CB * CB; e += 256) {
    const int r = e / CB, c = e % CB;
    if (r < nb && c <= r) A[(int64_t)(r0 + r) * m + r0 + c] = T[r][c];
  }
}

// Block row i = p + 1 + blockIdx.x: X L_pp^T = A_ip, one row of X per thread
// (the row lives in registers; L_pp is read from LDS by broadcast).
__global__ void __launch_bounds__(CB)
    chol_trsm_kernel(int m, int p, double* __restrict__ A) {
  __shared__ double L[CB][CBP];
  const int r0 = p * CB;
  const int i0 = (p + 1 + blockIdx.x) * CB;
  const int ni = min(CB, m - i0);
  const int np = min(CB, m - r0);
  for (int e = threadIdx.x; e < CB * CB; e += CB) {
    const int r = e / CB, c = e % CB;
    L[r][c] = (r < np && c < np) ? A[(int64_t)(r0 + r) * m + r0 + c] : (r == c ? 1.0 : 0.0);
  }
  __syncthreads();
  const int r = threadIdx.x;
  if (r >= ni) return;
  double* row = A + (int64_t)(i0 + r) * m + r0;
  double x[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) x[c] = c < np ? row[c] : 0.0;
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    double v = x[c];
#pragma unroll
    for (int t = 0; t < c; ++t) v -= x[t] * L[c][t];
    x[c] = v / L[c][c];
  }
#pragma unroll
  for (int c = 0; c < CB; ++c)
    if (c < np) row[c] = x[c];
}

// Trailing update of block (i, j), p < j <= i, enumerated row by row. Both
// panels are staged transposed (dynamic LDS, 2 x 64 x 65 doubles) so that
// the inner loop reads consecutive words; thread (tx, ty) owns rows ty + 16 q
// and columns tx + 16 w of the block.
__global__ void __launch_bounds__(256)
    chol_update_kernel(int m, int p, double* __restrict__ A) {
  extern __shared__ double lds[];
  double(*LiT)[CBP] = reinterpret_cast<double(*)[CBP]>(lds);
  double(*LjT)[CBP] = reinterpret_cast<double(*)[CBP]>(lds + CB * CBP);
  // blockIdx.x -> (ii, jj) with 0 <= jj <= ii over the trailing blocks
  int ii = 0, rem = blockIdx.x;
  while (rem > ii) {
    rem -= ii + 1;
    ++ii;
  }
  const int jj = rem;
  const int i0 = (p + 1 + ii) * CB, j0 = (p + 1 + jj) * CB, c0 = p * CB;
  const int ni = min(CB, m - i0), nj = min(CB, m - j0), nc = min(CB, m - c0);
  for (int e = threadIdx.x; e < CB * CB; e += 256) {
    const int r = e / CB, c = e % CB;
    LiT[c][r] = (r < ni && c < nc) ? A[(int64_t)(i0 + r) * m + c0 + c] : 0.0;
    LjT[c][r] = (r < nj && c < nc) ? A[(int64_t)(j0 + r) * m + c0 + c] : 0.0;
  }
  __syncthreads();
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  for (int t = 0; t < CB; ++t) {
    double a[4], bb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = LiT[t][ty + 16 * q];
      bb[q] = LjT[t][tx + 16 * q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int w = 0; w < 4; ++w) acc[q][w] = __builtin_fma(a[q], bb[w], acc[q][w]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int r = ty + 16 * q, c = tx + 16 * w;
      if (r < ni && c < nj && (ii != jj || c <= r)) A[(int64_t)(i0 + r) * m + j0 + c] -= acc[q][w];
    }
}

// L L^T x = b by blocks of 64 in one workgroup; x scattered to d[idx].
__global__ void __launch_bounds__(1024)
    chol_solve_kernel(int m, const double* __restrict__ A, double* __restrict__ b,
                      const int* __restrict__ idx, double* __restrict__ d,
                      const int* __restrict__ ok) {
  if (*ok == 0) return;
  __shared__ double y[CB];
  const int tid = threadIdx.x;
  const int T = (m + CB - 1) / CB;
  // forward: L y = b
  for (int bp = 0; bp < T; ++bp) {
    const int r0 = bp * CB, nb = min(CB, m - r0);
    if (tid < 64) {
      double v = tid < nb ? b[r0 + tid] : 0.0;
      for (int c = 0; c < nb; ++c) {
        const double yc = __shfl(v, c, 64) / A[(int64_t)(r0 + c) * m + r0 + c];
        if (tid == c) v = yc;
        if (tid > c && tid < nb) v -= A[(int64_t)(r0 + tid) * m + r0 + c] * yc;
      }
      if (tid < nb) {
        y[tid] = v;
        b[r0 + tid] = v;
      }
    }
    __syncthreads();
    for (int i = r0 + nb + tid; i < m; i += 1024) {
      double v = b[i];
      const double* Li = A + (int64_t)i * m + r0;
      for (int c = 0; c < nb; ++c) v -= Li[c] * y[c];
      b[i] = v;
    }
    __syncthreads();
  }
  // backward: L^T x = y
  for (int bp = T - 1; bp >= 0; --bp) {
    const int r0 = bp * CB, nb = min(CB, m - r0);
    if (tid < 64) {
      double v = tid < nb ? b[r0 + tid] : 0.0;
      for (int c = nb - 1; c >= 0; --c) {
        const double xc = __shfl(v, c, 64) / A[(int64_t)(r0 + c) * m + r0 + c];
        if (tid == c) v = xc;
        if (tid < c) v -= A[(int64_t)(r0 + c) * m + r0 + tid] * xc;
      }
      if (tid < nb) {
        y[tid] = v;
        b[r0 + tid] = v;
      }
    }
    __syncthreads();
    for (int i = tid; i < r0; i += 1024) {
      double v = b[i];
      for (int c = 0; c < nb; ++c) v -= A[(int64_t)(r0 + c) * m + i] * y[c];
      b[i] = v;
    }
    __syncthreads();
  }
  for (int a = tid; a < m; a += 1024) d[idx[a]] = b[a];
}

__global__ void set_ok_kernel(int* ok) { *ok = 1; }

hipError_t launch_newton_direction_blocked(hipStream_t s, int K, int m, const int64_t* Nk,
                                           const double* H, const double* S, double* A,
                                           const int* idx, double* d, int* ok) {
  double* b = A + (int64_t)m * m;
  const int64_t tot = std::max<int64_t>((int64_t)m * m, K);
  hipLaunchKernelGGL(reduced_gather_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     K, m, idx, H, S, Nk, A, b, d);
  hipLaunchKernelGGL(set_ok_kernel, dim3(1), dim3(1), 0, s, ok);
  const int T = (m + CB - 1) / CB;
  const size_t upd_lds = sizeof(double) * 2 * CB * CBP;
  static const bool attr = [] {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_update_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(double) * 2 * CB * CBP)) != hipSuccess)
      (void)hipGetLastError();  // clear; a launch that still fails reports it
    return true;
  }();
  (void)attr;
  for (int p = 0; p < T; ++p) {
    hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, s, m, p, A, ok);
    const int rest = T - p - 1;
    if (rest > 0) {
      hipLaunchKernelGGL(chol_trsm_kernel, dim3(rest), dim3(CB), 0, s, m, p, A);
      hipLaunchKernelGGL(chol_update_kernel, dim3(rest * (rest + 1) / 2), dim3(256), upd_lds, s,
                         m, p, A);
    }
  }
  hipLaunchKernelGGL(chol_solve_kernel, dim3(1), dim3(1024), 0, s, m, A, b, idx, d, ok);
  return hipGetLastError();
}

}  // namespace bumbar
