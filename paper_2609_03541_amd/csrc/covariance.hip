// Asymptotic covariance of the free energies f (the large-sample covariance
// of the MBAR estimate, Shirts and Chodera, J. Chem. Phys. 129, 124105
// (2008); the paper names uncertainty estimates as related work in
// Section 1). With W_nk = exp(f_k - u_kn - ln D_n) at the solution,
//   Theta = W^T (I_N - W diag(N) W^T)^+ W,  Cov(f_i, f_j) = (e_i - e_0)^T Theta (e_j - e_0).
// The N x N pseudo-inverse reduces to K x K algebra: with M = W^T W, the
// sampled states S and B = diag(N_S) M_{S,:},
//   Theta = M + B^T G B - 1 1^T / N_tot,
// G any generalised inverse of H_S = diag(N_S) - diag(N_S) M_SS diag(N_S),
// the Hessian of the objective on the sampled states; the last term drops
// out of every contrast. G = H_red^{-1} on all sampled states but the first
// (zero on that one), and H_red = L L^T, so B^T G B = Z^T Z with
// Z = L^{-1} B_red. The steps:
//   M      the Hessian contraction (FP64 matrix cores) with P = W, i.e.
//          constants c_k = f_k and unit scales, and S = 0: it returns -M;
//   gather H_red and B_red = diag(N) M over the kept states;
//   factor H_red by the blocked Cholesky of the Newton finisher;
//   Z      block forward substitution, Z_p = L_pp^{-1} (B_p - sum_q<p L_pq Z_q);
//   Theta  M + Z^T Z (64 x 64 output tiles, FP64 FMA);
//   Cov    the contrasts against state 0.
#include <algorithm>
#include <cmath>

#include "bumbar_impl.h"

namespace bumbar {

constexpr int VB = 64;       // tile edge
constexpr int VBP = VB + 1;  // padded LDS row
constexpr int VT = 256;      // threads (16 x 16), each owning a 4 x 4 sub-tile

__global__ void cov_consts_kernel(int K, const double* __restrict__ f, double* __restrict__ cst,
                                  double* __restrict__ gk, double* __restrict__ S) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) {
    cst[k] = f[k];
    gk[k] = 1.0;
    S[k] = 0.0;
  }
}

// A (m x m) = H_red, Bm (m x K) = N_r M_rj over the kept states idx, b = 0;
// Mneg = -M.
__global__ void cov_gather_kernel(int K, int m, const int* __restrict__ idx,
                                  const int64_t* __restrict__ Nk, const double* __restrict__ Mneg,
                                  double* __restrict__ A, double* __restrict__ b,
                                  double* __restrict__ Bm) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < (int64_t)m * m) {
    const int r = (int)(e / m), c = (int)(e % m);
    const double nr = (double)Nk[idx[r]], nc = (double)Nk[idx[c]];
    A[e] = (r == c ? nr : 0.0) + nr * nc * Mneg[(int64_t)idx[r] * K + idx[c]];
  }
  if (e < (int64_t)m * K) {
    const int r = (int)(e / K), j = (int)(e % K);
    Bm[e] = -(double)Nk[idx[r]] * Mneg[(int64_t)idx[r] * K + j];
  }
  if (e < m) b[e] = 0.0;
}

// Z_p = L_pp^{-1} R_p in place over block row p of Bm (rows p*64 ...), one
// workgroup per 64-column tile. Linv_p is lower triangular; rows of R past m
// are taken as zero.
__global__ void __launch_bounds__(VT)
    cov_fwd_diag_kernel(int m, int K, int p, const double* __restrict__ Linv,
                        double* __restrict__ Bm) {
  __shared__ double Ls[VB][VBP];  // Ls[i][t] = Linv_p[i][t]
  __shared__ double Rs[VB][VBP];  // Rs[t][c]
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int r0 = p * VB, c0 = blockIdx.x * VB;
  const int nb = min(VB, m - r0), nc = min(VB, K - c0);
  const double* Lp = Linv + (int64_t)p * VB * VB;
  for (int e = tid; e < VB * VB; e += VT) {
    const int a = e >> 6, c = e & (VB - 1);
    Ls[a][c] = Lp[e];
    Rs[a][c] = (a < nb && c < nc) ? Bm[(int64_t)(r0 + a) * K + c0 + c] : 0.0;
  }
  __syncthreads();
  double acc[4][4] = {};
  for (int t = 0; t < nb; ++t) {
    double l[4], r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) l[q] = Ls[ty + 16 * q][t];
#pragma unroll
    for (int w = 0; w < 4; ++w) r[w] = Rs[t][tx + 16 * w];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int w = 0; w < 4; ++w) acc[q][w] = __builtin_fma(l[q], r[w], acc[q][w]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int i = ty + 16 * q, c = tx + 16 * w;
      if (i < nb && c < nc) Bm[(int64_t)(r0 + i) * K + c0 + c] = acc[q][w];
    }
}

// Bm_i -= L_ip Z_p for the block rows i > p: blockIdx.y picks i, blockIdx.x
// the 64-column tile. L_ip is the lower block (i, p) of the factored matrix
// (full 64 columns, since p is not the last block).
__global__ void __launch_bounds__(VT)
    cov_fwd_update_kernel(int m, int K, int p, const double* __restrict__ A,
                          double* __restrict__ Bm) {
  __shared__ double Ls[VB][VBP];  // Ls[r][t] = L_ip[r][t]
  __shared__ double Zs[VB][VBP];  // Zs[t][c] = Z_p[t][c]
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int p0 = p * VB, i0 = (p + 1 + (int)blockIdx.y) * VB, c0 = blockIdx.x * VB;
  const int ni = min(VB, m - i0), nc = min(VB, K - c0);
  for (int e = tid; e < VB * VB; e += VT) {
    const int a = e >> 6, c = e & (VB - 1);
    Ls[a][c] = a < ni ? A[(int64_t)(i0 + a) * m + p0 + c] : 0.0;
    Zs[a][c] = c < nc ? Bm[(int64_t)(p0 + a) * K + c0 + c] : 0.0;
  }
  __syncthreads();
  double acc[4][4] = {};
  for (int t = 0; t < VB; ++t) {
    double l[4], z[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) l[q] = Ls[ty + 16 * q][t];
#pragma unroll
    for (int w = 0; w < 4; ++w) z[w] = Zs[t][tx + 16 * w];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int w = 0; w < 4; ++w) acc[q][w] = __builtin_fma(l[q], z[w], acc[q][w]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int r = ty + 16 * q, c = tx + 16 * w;
      if (r < ni && c < nc) Bm[(int64_t)(i0 + r) * K + c0 + c] -= acc[q][w];
    }
}

// Theta = -Mneg + Z^T Z (Z m x K), one workgroup per 64 x 64 output tile,
// the m rows of Z taken 64 at a time through LDS.
__global__ void __launch_bounds__(VT)
    cov_theta_kernel(int m, int K, const double* __restrict__ Z, const double* __restrict__ Mneg,
                     double* __restrict__ Th) {
  __shared__ double Zi[VB][VBP];  // Zi[t][i] = Z[t0 + t][i0 + i]
  __shared__ double Zj[VB][VBP];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.y * VB, j0 = blockIdx.x * VB;
  const int ni = min(VB, K - i0), nj = min(VB, K - j0);
  double acc[4][4] = {};
  for (int t0 = 0; t0 < m; t0 += VB) {
    const int nt = min(VB, m - t0);
    __syncthreads();
    for (int e = tid; e < VB * VB; e += VT) {
      const int t = e >> 6, c = e & (VB - 1);
      const double* row = Z + (int64_t)(t0 + t) * K;
      Zi[t][c] = (t < nt && c < ni) ? row[i0 + c] : 0.0;
      Zj[t][c] = (t < nt && c < nj) ? row[j0 + c] : 0.0;
    }
    __syncthreads();
    for (int t = 0; t < nt; ++t) {
      double a[4], g[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = Zi[t][ty + 16 * q];
#pragma unroll
      for (int w = 0; w < 4; ++w) g[w] = Zj[t][tx + 16 * w];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[q][w] = __builtin_fma(a[q], g[w], acc[q][w]);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int i = ty + 16 * q, j = tx + 16 * w;
      if (i < ni && j < nj) {
        const int64_t o = (int64_t)(i0 + i) * K + j0 + j;
        Th[o] = acc[q][w] - Mneg[o];
      }
    }
}

// Cov_ij = Theta_ij - Theta_i0 - Theta_0j + Theta_00; exactly zero on row
// and column 0 (f_0 is fixed by the gauge).
__global__ void cov_gauge_kernel(int K, const double* __restrict__ Th, double* __restrict__ cov) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)K * K) return;
  const int i = (int)(e / K), j = (int)(e % K);
  cov[e] = (i == 0 || j == 0) ? 0.0
                              : ((Th[e] - Th[(int64_t)i * K]) - Th[j]) + Th[0];
}

hipError_t launch_cov_consts(hipStream_t s, int K, const double* f, double* cst, double* gk,
                             double* S) {
  hipLaunchKernelGGL(cov_consts_kernel, dim3((K + 255) / 256), dim3(256), 0, s, K, f, cst, gk, S);
  return hipGetLastError();
}

hipError_t launch_cov_gather(hipStream_t s, int K, int m, const int* idx, const int64_t* Nk,
                             const double* Mneg, double* A, double* b, double* Bm) {
  const int64_t tot = std::max<int64_t>(std::max<int64_t>((int64_t)m * m, (int64_t)m * K), 1);
  hipLaunchKernelGGL(cov_gather_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, K, m,
                     idx, Nk, Mneg, A, b, Bm);
  return hipGetLastError();
}

hipError_t launch_cov_solve(hipStream_t s, int m, int K, const double* A, const double* Linv,
                            double* Bm) {
  const int T = (m + VB - 1) / VB;
  const unsigned ct = (unsigned)((K + VB - 1) / VB);
  for (int p = 0; p < T; ++p) {
    hipLaunchKernelGGL(cov_fwd_diag_kernel, dim3(ct), dim3(VT), 0, s, m, K, p, Linv, Bm);
    if (p + 1 < T)
      hipLaunchKernelGGL(cov_fwd_update_kernel, dim3(ct, (unsigned)(T - p - 1)), dim3(VT), 0, s, m,
                         K, p, A, Bm);
  }
  return hipGetLastError();
}

hipError_t launch_cov_theta(hipStream_t s, int m, int K, const double* Z, const double* Mneg,
                            double* Th, double* cov) {
  const unsigned ct = (unsigned)((K + VB - 1) / VB);
  hipLaunchKernelGGL(cov_theta_kernel, dim3(ct, ct), dim3(VT), 0, s, m, K, Z, Mneg, Th);
  const int64_t kk = (int64_t)K * K;
  hipLaunchKernelGGL(cov_gauge_kernel, dim3((unsigned)((kk + 255) / 256)), dim3(256), 0, s, K, Th,
                     cov);
  return hipGetLastError();
}

}  // namespace bumbar
