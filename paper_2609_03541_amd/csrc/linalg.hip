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
// right-looking Cholesky factorisation A = L L^T (64 x 64 blocks) with the
// forward substitution L y = b folded in, then a backward substitution
// L^T x = y. Each diagonal block L_pp is factored in LDS together with its
// inverse, so that the blocks below it, L_ip = A_ip L_pp^{-T}, and the piece
// y_p = L_pp^{-1} b_p are products rather than serial substitutions.
//
// Per block column p one launch (chol_step_kernel) covers every trailing block
// (i, j), p < j <= i: it forms L_ip and L_jp from the untouched A_ip, A_jp and
// subtracts L_ip L_jp^T from A_ij; the diagonal blocks (i, i) also store
// L_ip^T in the upper block (p, i) (the lower one is still read by other
// workgroups of the launch) and take b_i -= L_ip y_p; the workgroup of block
// (p+1, p+1), whose update is the last that block receives, factors it
// straight away for the next launch. Storage after the factorisation: the
// diagonal blocks hold L_pp below and L_pp^T above the diagonal, the upper
// off-diagonal blocks hold L^T (copied to the lower ones before the backward
// substitution), and the inverses L_pp^{-1} sit in a separate array. A pivot
// that is not positive clears *ok, as in the LDS kernel; the launches after
// it return at once.
namespace bumbar {

constexpr int CB = 64;       // Cholesky block edge
constexpr int CBP = CB + 1;  // padded LDS row
constexpr int CT = 256;      // threads of the factorisation kernels (16 x 16)

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

// Factorisation of one 64 x 64 diagonal block held in registers: thread
// (tx, ty) of 16 x 16 owns t[q][w] = T[ty + 16 q][tx + 16 w] (padding rows and
// columns hold the identity; only the lower triangle is read). L D L^T first
// (unit lower L', no square roots): at step j every A_ik, j < k <= i, loses
// A_ij A_kj / A_jj, and Y = L'^{-1} is built alongside by the same column (row
// i of Y loses L'_ij times row j). Column j of T and row j of Y are final at
// step j; their owners publish them to a double-buffered LDS vector, one
// barrier per column. Then L = L' D^{1/2} and L^{-1} = D^{-1/2} L'^{-1}: on
// return t holds L (zero above the diagonal) and y holds L^{-1}. Returns
// false, uniformly, on a pivot that is not positive. lds: 5 * 64 doubles.
__device__ bool factor_regs(double (&t)[4][4], double (&y)[4][4], double* lds) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double* cb = lds;           // [2][64] column j of T
  double* yb = lds + 2 * CB;  // [2][64] row j of Y
  double* sd = lds + 4 * CB;  // sqrt(D)
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) y[q][w] = (ty + 16 * q == tx + 16 * w) ? 1.0 : 0.0;
#pragma unroll
  for (int wj = 0; wj < 4; ++wj) {
#pragma unroll 1
    for (int tj = 0; tj < 16; ++tj) {
      const int j = 16 * wj + tj;
      double* cj = cb + (j & 1) * CB;
      double* yj = yb + (j & 1) * CB;
      if (tx == tj) {
#pragma unroll
        for (int q = 0; q < 4; ++q) cj[ty + 16 * q] = t[q][wj];
      }
      if (ty == tj) {
#pragma unroll
        for (int w = 0; w < 4; ++w) yj[tx + 16 * w] = y[wj][w];
      }
      __syncthreads();
      const double piv = cj[j];
      if (!(piv > 0.0)) return false;
      const double rp = 1.0 / piv;
      // rows i <= j and the columns each update must not touch take a zero
      // factor (every operand is finite, so x - 0 * v = x exactly)
      double li[4], ck[4], yc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) li[q] = ty + 16 * q > j ? -cj[ty + 16 * q] * rp : 0.0;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const bool right = tx + 16 * w > j;
        ck[w] = right ? cj[tx + 16 * w] : 0.0;
        yc[w] = right ? 0.0 : yj[tx + 16 * w];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          t[q][w] = __builtin_fma(li[q], ck[w], t[q][w]);
          y[q][w] = __builtin_fma(li[q], yc[w], y[q][w]);
        }
    }
  }
  if (tx == ty) {
#pragma unroll
    for (int q = 0; q < 4; ++q) sd[tx + 16 * q] = sqrt(t[q][q]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int i = ty + 16 * q, k = tx + 16 * w;
      t[q][w] = k < i ? t[q][w] / sd[k] : (k == i ? sd[i] : 0.0);
      y[q][w] = k <= i ? y[q][w] / sd[i] : 0.0;
    }
  return true;
}

// Factor the diagonal block at rows/columns r0 .. r0+nb-1 (t as in
// factor_regs), store L below and L^T above its diagonal in A, L^{-1}
// (64 x 64, row-major, zero above the diagonal) in Linv_blk and, for the last
// block, y = L^{-1} bv. Ls: a 64 x 65 LDS tile (the transpose), lds: 5 * 64
// doubles.
__device__ void finish_diag(double (&t)[4][4], double (*Ls)[CBP], double* lds, const double* bv,
                            int nb, int r0, bool last, int m, double* __restrict__ A,
                            double* __restrict__ Linv_blk, double* __restrict__ y,
                            int* __restrict__ ok) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double yi[4][4];
  if (!factor_regs(t, yi, lds)) {
    if (tid == 0) *ok = 0;
    return;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      Ls[ty + 16 * q][tx + 16 * w] = t[q][w];
      Linv_blk[(ty + 16 * q) * CB + tx + 16 * w] = yi[q][w];
    }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int i = ty + 16 * q, k = tx + 16 * w;
      if (i < nb && k < nb) A[(int64_t)(r0 + i) * m + r0 + k] = k <= i ? t[q][w] : Ls[k][i];
    }
  if (last) {
    // y_i = sum_c L^{-1}_ic b_c: partial sums over the thread's columns, then
    // over the 16 threads that share its rows (lanes tx of one wave)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < 4; ++w) v = __builtin_fma(yi[q][w], bv[tx + 16 * w], v);
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 16);
      const int i = ty + 16 * q;
      if (tx == 0 && i < nb) y[r0 + i] = v;
    }
  }
}

// The first diagonal block (one workgroup).
__global__ void __launch_bounds__(CT)
    chol_first_kernel(int m, double* __restrict__ A, const double* __restrict__ b,
                      double* __restrict__ y, double* __restrict__ Linv, int* __restrict__ ok) {
  __shared__ double Ls[CB][CBP];
  __shared__ double work[5 * CB];
  __shared__ double bv[CB];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int nb = min(CB, m);
  double t[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int i = ty + 16 * q, k = tx + 16 * w;
      t[q][w] = (i < nb && k < nb) ? A[(int64_t)i * m + k] : (i == k ? 1.0 : 0.0);
    }
  if (tid < CB) bv[tid] = tid < nb ? b[tid] : 0.0;
  __syncthreads();
  finish_diag(t, Ls, work, bv, nb, 0, m <= CB, m, A, Linv, y, ok);
}

// Block column p: one workgroup per trailing block (i, j), p < j <= i,
// enumerated row by row so that workgroup 0 owns block (p+1, p+1). Thread
// (tx, ty) owns rows ty + 16 q and columns tx + 16 w of each 64 x 64 product;
// operands sit in LDS transposed (element [t][r]) so the inner loops read
// consecutive words.
__global__ void __launch_bounds__(CT)
    chol_step_kernel(int m, int p, double* __restrict__ A, double* __restrict__ b,
                     double* __restrict__ y, double* __restrict__ Linv, int* __restrict__ ok) {
  if (*ok == 0) return;
  extern __shared__ double lds[];
  double(*S0)[CBP] = reinterpret_cast<double(*)[CBP]>(lds);
  double(*S1)[CBP] = reinterpret_cast<double(*)[CBP]>(lds + CB * CBP);
  double(*S2)[CBP] = reinterpret_cast<double(*)[CBP]>(lds + 2 * CB * CBP);
  double* bv = lds + 3 * CB * CBP;
  double* yv = bv + CB;
  int ii = 0, rem = blockIdx.x;
  while (rem > ii) {
    rem -= ii + 1;
    ++ii;
  }
  const int jj = rem;
  const bool dg = ii == jj;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int c0 = p * CB, i0 = c0 + (1 + ii) * CB, j0 = c0 + (1 + jj) * CB;
  const int ni = min(CB, m - i0), nj = min(CB, m - j0);
  const double* Lp = Linv + (int64_t)p * CB * CB;
  // S0[t][c] = Linv_p[c][t], S1[t][r] = A_ip[r][t], S2[t][r] = A_jp[r][t]
  for (int e = tid; e < CB * CB; e += CT) {
    const int r = e >> 6, c = e & (CB - 1);
    S0[c][r] = Lp[e];
    S1[c][r] = r < ni ? A[(int64_t)(i0 + r) * m + c0 + c] : 0.0;
    if (!dg) S2[c][r] = r < nj ? A[(int64_t)(j0 + r) * m + c0 + c] : 0.0;
  }
  if (dg && tid < CB) bv[tid] = b[c0 + tid];
  __syncthreads();
  // L_ip = A_ip Linv_p^T (and L_jp), and y_p = Linv_p b_p
  double li[4][4] = {}, lj[4][4] = {};
  for (int t = 0; t < CB; ++t) {
    double a[4], g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = S1[t][ty + 16 * q];
      g[q] = S0[t][tx + 16 * q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int w = 0; w < 4; ++w) li[q][w] = __builtin_fma(a[q], g[w], li[q][w]);
    if (!dg) {
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = S2[t][ty + 16 * q];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int w = 0; w < 4; ++w) lj[q][w] = __builtin_fma(a[q], g[w], lj[q][w]);
    }
  }
  if (dg && tid < CB) {
    double v = 0.0;
    for (int t = 0; t <= tid; ++t) v = __builtin_fma(S0[t][tid], bv[t], v);
    yv[tid] = v;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      S1[tx + 16 * w][ty + 16 * q] = li[q][w];
      if (!dg) S2[tx + 16 * w][ty + 16 * q] = lj[q][w];
    }
  __syncthreads();
  double(*LjT)[CBP] = dg ? S1 : S2;
  double acc[4][4] = {};
  for (int t = 0; t < CB; ++t) {
    double a[4], g[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = S1[t][ty + 16 * q];
      g[q] = LjT[t][tx + 16 * q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int w = 0; w < 4; ++w) acc[q][w] = __builtin_fma(a[q], g[w], acc[q][w]);
  }
  const bool fac = dg && ii == 0;
  if (dg) {
    // upper block (p, i) = L_ip^T, and b_i -= L_ip y_p
    for (int e = tid; e < CB * CB; e += CT) {
      const int t = e >> 6, r = e & (CB - 1);
      if (r < ni) A[(int64_t)(c0 + t) * m + i0 + r] = S1[t][r];
    }
    if (tid < CB) {
      double v = 0.0;
      if (tid < ni) {
        for (int t = 0; t < CB; ++t) v = __builtin_fma(S1[t][tid], yv[t], v);
        v = b[i0 + tid] - v;
        b[i0 + tid] = v;
      }
      if (ii == 0) y[c0 + tid] = yv[tid];
      if (fac) bv[tid] = v;  // b_{p+1} is final now
    }
  }
  if (!fac) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int r = ty + 16 * q, c = tx + 16 * w;
        if (r < ni && c < nj && (!dg || c <= r)) A[(int64_t)(i0 + r) * m + j0 + c] -= acc[q][w];
      }
    return;
  }
  // block (p+1, p+1) has received its last update: factor it
  __syncthreads();
  double tt[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int r = ty + 16 * q, c = tx + 16 * w;
      tt[q][w] = (r < ni && c < ni) ? A[(int64_t)(i0 + r) * m + i0 + c] - acc[q][w]
                                    : (r == c ? 1.0 : 0.0);
    }
  finish_diag(tt, S1, S2[0], bv, ni, i0, i0 + CB >= m, m, A, Linv + (int64_t)(p + 1) * CB * CB, y,
              ok);
}

// After the factorisation the off-diagonal blocks of L sit transposed in the
// upper triangle; this copies each one, upper block (p, i) = L_ip^T, back to
// the lower block (i, p) through an LDS tile, so that the backward
// substitution reads L by rows. One workgroup per block, (i, p) enumerated
// row by row.
__global__ void __launch_bounds__(CT)
    chol_mirror_kernel(int m, double* __restrict__ A, const int* __restrict__ ok) {
  if (*ok == 0) return;
  __shared__ double tile[CB][CBP];
  int ii = 1, rem = blockIdx.x;
  while (rem >= ii) {
    rem -= ii;
    ++ii;
  }
  const int i0 = ii * CB, p0 = rem * CB;
  const int ni = min(CB, m - i0);
  const int tid = threadIdx.x;
  for (int e = tid; e < CB * CB; e += CT) {
    const int t = e >> 6, r = e & (CB - 1);
    if (r < ni) tile[t][r] = A[(int64_t)(p0 + t) * m + i0 + r];
  }
  __syncthreads();
  for (int e = tid; e < CB * CB; e += CT) {
    const int r = e >> 6, t = e & (CB - 1);
    if (r < ni) A[(int64_t)(i0 + r) * m + p0 + t] = tile[t][r];
  }
}

// L^T x = y in one workgroup, block by block from the last: x_p = L_pp^{-T} z_p
// (L_pp^{-1} staged in LDS, the 64 x 64 product split over all threads), then
// z_i -= sum_c L[r0 + c][i] x_c for every row i above the block: thread i
// reads column i of the block's rows of L, so the loads of a wave are
// consecutive and each thread has its 64 loads in flight together. z starts
// as y and ends as x, which is scattered to d[idx].
constexpr int BT = 512;  // threads of the backward substitution (8 waves)
constexpr int BW = BT / 64;

__global__ void __launch_bounds__(BT)
    chol_back_kernel(int m, const double* __restrict__ A, const double* __restrict__ y,
                     const double* __restrict__ Linv, double* __restrict__ z,
                     const int* __restrict__ idx, double* __restrict__ d,
                     const int* __restrict__ ok) {
  if (*ok == 0) return;
  __shared__ double Lt[CB][CBP];
  __shared__ double part[BW][CB];
  __shared__ double zb[CB];
  __shared__ double xs[CB];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int T = (m + CB - 1) / CB;
  for (int i = tid; i < m; i += BT) z[i] = y[i];
  __syncthreads();
  for (int bp = T - 1; bp >= 0; --bp) {
    const int r0 = bp * CB, nb = min(CB, m - r0);
    const double* Lb = Linv + (int64_t)bp * CB * CB;
    for (int e = tid; e < CB * CB; e += BT) Lt[e >> 6][e & (CB - 1)] = Lb[e];
    if (tid < CB) zb[tid] = tid < nb ? z[r0 + tid] : 0.0;
    __syncthreads();
    {
      // x_c = sum_t Linv[t][c] z_t; wave g takes 8 consecutive t
      constexpr int TG = CB / BW;
      double v = 0.0;
#pragma unroll
      for (int t = TG * wv; t < TG * wv + TG; ++t) v = __builtin_fma(Lt[t][lane], zb[t], v);
      part[wv][lane] = v;
    }
    __syncthreads();
    if (tid < CB) {
      double v = 0.0;
#pragma unroll
      for (int g = 0; g < BW; ++g) v += part[g][tid];
      xs[tid] = v;
      if (tid < nb) z[r0 + tid] = v;
    }
    __syncthreads();
    for (int i = tid; i < r0; i += BT) {
      const double* col = A + (int64_t)r0 * m + i;
      double v = 0.0;
      if (nb == CB) {
#pragma unroll
        for (int h = 0; h < CB; h += 32) {
          double a[32];
#pragma unroll
          for (int c = 0; c < 32; ++c) a[c] = col[(int64_t)(h + c) * m];
#pragma unroll
          for (int c = 0; c < 32; ++c) v = __builtin_fma(a[c], xs[h + c], v);
        }
      } else {
        for (int c = 0; c < nb; ++c) v = __builtin_fma(col[(int64_t)c * m], xs[c], v);
      }
      z[i] -= v;
    }
    __syncthreads();
  }
  for (int a = tid; a < m; a += BT) d[idx[a]] = z[a];
}

__global__ void set_ok_kernel(int* ok) { *ok = 1; }

size_t newton_ws_doubles(int K) {
  return (size_t)K * K + 3 * (size_t)K + (size_t)((K + CB - 1) / CB) * CB * CB;
}

hipError_t launch_chol_factor_blocked(hipStream_t s, int m, double* A, double* b, double* y,
                                     double* Linv, int* ok) {
  if (m <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(set_ok_kernel, dim3(1), dim3(1), 0, s, ok);
  const size_t step_lds = sizeof(double) * (3 * CB * CBP + 2 * CB);
  static const bool attr = [&] {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_step_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)step_lds) != hipSuccess)
      (void)hipGetLastError();  // clear; a launch that still fails reports it
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL(chol_first_kernel, dim3(1), dim3(CT), 0, s, m, A, b, y, Linv, ok);
  const int T = (m + CB - 1) / CB;
  for (int p = 0; p + 1 < T; ++p) {
    const int rest = T - p - 1;
    hipLaunchKernelGGL(chol_step_kernel, dim3(rest * (rest + 1) / 2), dim3(CT), step_lds, s, m, p,
                       A, b, y, Linv, ok);
  }
  if (T > 1)
    hipLaunchKernelGGL(chol_mirror_kernel, dim3(T * (T - 1) / 2), dim3(CT), 0, s, m, A, ok);
  return hipGetLastError();
}

hipError_t launch_newton_direction_blocked(hipStream_t s, int K, int m, const int64_t* Nk,
                                           const double* H, const double* S, double* A,
                                           const int* idx, double* d, int* ok) {
  if (m <= 0 || m >= K) return hipErrorInvalidValue;
  double* b = A + (int64_t)m * m;
  double* y = b + m;
  double* Linv = y + m;
  const int64_t tot = std::max<int64_t>((int64_t)m * m, K);
  hipLaunchKernelGGL(reduced_gather_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     K, m, idx, H, S, Nk, A, b, d);
  const hipError_t e = launch_chol_factor_blocked(s, m, A, b, y, Linv, ok);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(chol_back_kernel, dim3(1), dim3(BT), 0, s, m, A, y, Linv, b, idx, d, ok);
  return hipGetLastError();
}

}  // namespace bumbar
