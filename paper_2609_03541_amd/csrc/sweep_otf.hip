// Sweeps with the reduced energies computed on the fly from the bias model
// (Section 2: the energies of umbrella windows are known functions of the
// sampled coordinate; any potential common to all states cancels in Eq. (1)
// and is left out). u_kn is never stored: each kernel reads the N x d
// coordinates and the K model coefficients and evaluates
//   HARMONIC  u_k(x) = a_k + sum_j kappa_kj / 2 (x_j - x0_kj)^2
//   LINEAR    u_k(x) = a_k + sum_j b_kj x_j
// per element, so the sweep is bound by arithmetic (exponentials), not HBM.
//
// Two passes, as for large K with a stored matrix: a column pass (exact
// log-sum-exp over sampled states per sample, online max in chunks of 8
// states with the state coefficients staged in LDS tiles) and a state pass
// (each thread accumulates 8 or 16 states over a strided set of samples;
// per-block partials are written state-major for the common finaliser).
//
// FP64 kernels evaluate u in the direct form above from FP64 coordinates and
// use the FP64 exponential. FP32 kernels (mixed precision) use the expanded
// quadratic form t = A_k + sum_j (B_kj x_j + C_kj x_j^2) in log2 units with
// the hardware exp2, from FP32 coordinates; A, B, C are rebuilt in FP64 for
// every sweep and rounded once.
#include <algorithm>
#include <cmath>

#include "bumbar_impl.h"
#include "devmath.h"

namespace bumbar {

constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;
constexpr int kOT = 256;        // threads per block (both passes)
constexpr int kOTile = 512;     // states per LDS tile in the column pass
constexpr int kOStates = 64;    // states per state-pass block (4 row groups)

int otf_grid(int64_t N, int num_cus) {
  int64_t g = (N + 2 * kOT - 1) / (2 * kOT);
  const int64_t cap = (int64_t)num_cus * 4;
  if (g > cap) g = cap;
  if (g > sweep_max_grid(num_cus)) g = sweep_max_grid(num_cus);
  return (int)(g < 1 ? 1 : g);
}

// ---- coefficient preparation ------------------------------------------------

// FP32 coefficients in log2 units: cf = [A_col K | A_st K | B K*d | C K*d] with
// A_st = log2e (c_k - w0_k), A_col = A_st for sampled states and -inf
// otherwise, B = -log2e w1, C = -log2e w2, where u_k = w0 + sum (w1 x + w2 x^2).
__global__ void otf32_coef_kernel(int K, int d, int model, const double* __restrict__ coef,
                                  const double* __restrict__ cst, const double* __restrict__ gk,
                                  float* __restrict__ cf) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double* ck = coef + (int64_t)k * (1 + 2 * d);
  double w0 = ck[0];
  for (int j = 0; j < d; ++j) {
    double w1, w2;
    if (model == BUMBAR_MODEL_HARMONIC) {
      const double h = 0.5 * ck[1 + 2 * j], x0 = ck[2 + 2 * j];
      w0 += h * x0 * x0;
      w1 = -2.0 * h * x0;
      w2 = h;
    } else {
      w1 = ck[1 + j];
      w2 = 0.0;
    }
    cf[2 * K + (int64_t)j * K + k] = (float)(-kLog2e * w1);
    cf[2 * K + (int64_t)(d + j) * K + k] = (float)(-kLog2e * w2);
  }
  const float a = (float)(kLog2e * (cst[k] - w0));
  cf[K + k] = a;
  cf[k] = gk[k] != 0.0 ? a : -INFINITY;
}

// FP64 coefficients: c64 = [E_col K | E_st K | H K*d | X0 K*d] with
// E_st = c_k - a_k, E_col = E_st for sampled states and -inf otherwise (the
// column pass skips unsampled states); for HARMONIC, H = kappa / 2 and X0 =
// the centre; for LINEAR, H = b and X0 = 0 (the kernels branch on the model
// at compile time).
__global__ void otf64_coef_kernel(int K, int d, int model, const double* __restrict__ coef,
                                  const double* __restrict__ cst, const double* __restrict__ gk,
                                  double* __restrict__ c64) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double* ck = coef + (int64_t)k * (1 + 2 * d);
  for (int j = 0; j < d; ++j) {
    if (model == BUMBAR_MODEL_HARMONIC) {
      c64[2 * K + (int64_t)j * K + k] = 0.5 * ck[1 + 2 * j];
      c64[2 * K + (int64_t)(d + j) * K + k] = ck[2 + 2 * j];
    } else {
      c64[2 * K + (int64_t)j * K + k] = ck[1 + j];
      c64[2 * K + (int64_t)(d + j) * K + k] = 0.0;
    }
  }
  const double e = cst[k] - ck[0];
  c64[K + k] = e;
  c64[k] = gk[k] != 0.0 ? e : -INFINITY;
}

__global__ void pack_coords_kernel(int64_t n, const double* __restrict__ xi, float* __restrict__ xf) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) xf[i] = (float)xi[i];
}

// ---- model evaluation ---------------------------------------------------------

// sum_j H_j (x_j - X0_j)^2 (HARMONIC) or sum_j H_j x_j (LINEAR), FP64.
template <int D, int MODEL>
__device__ __forceinline__ double model_rest(const double* h, const double* x0, const double* x) {
  double q = 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    if (MODEL == BUMBAR_MODEL_HARMONIC) {
      const double dx = x[j] - x0[j];
      q = __builtin_fma(h[j] * dx, dx, q);
    } else {
      q = __builtin_fma(h[j], x[j], q);
    }
  }
  return q;
}

// ---- FP32 passes ----------------------------------------------------------------

template <int D>
__global__ void __launch_bounds__(kOT)
    otf32_colpass_kernel(int K, int64_t N, const float* __restrict__ xf,
                         const float* __restrict__ cf, const double* __restrict__ h,
                         double* __restrict__ logD,
                         double* __restrict__ part_obj, unsigned* __restrict__ part_flags) {
  __shared__ float sA[kOTile];
  __shared__ float sB[D][kOTile];
  __shared__ float sC[D][kOTile];
  __shared__ double wred[kOT / 64];
  __shared__ unsigned fl;
  if (threadIdx.x == 0) fl = 0u;
  double obj = 0.0;
  unsigned bad = 0;
  const int64_t stride = (int64_t)gridDim.x * kOT * 2;
  // every thread of the block runs the same number of column iterations (the
  // LDS tiles are shared), with out-of-range columns masked
  const int64_t n_iter = (N + stride - 1) / stride;
  for (int64_t it = 0; it < n_iter; ++it) {
    const int64_t n0 = it * stride + ((int64_t)blockIdx.x * kOT + threadIdx.x) * 2;
    const bool ok0 = n0 < N, ok1 = n0 + 1 < N;
    float x0[D], x1[D], q0[D], q1[D];
    float chk = 0.f;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      x0[j] = ok0 ? xf[n0 * D + j] : 0.f;
      x1[j] = ok1 ? xf[(n0 + 1) * D + j] : x0[j];
      q0[j] = x0[j] * x0[j];
      q1[j] = x1[j] * x1[j];
      chk += x0[j] + x1[j];
    }
    if (chk != chk) bad |= FLAG_NAN;
    float m0 = -1e30f, m1 = -1e30f, s0 = 0.f, s1 = 0.f;
    for (int t0 = 0; t0 < K; t0 += kOTile) {
      const int tl = min(kOTile, K - t0);
      __syncthreads();
      for (int i = threadIdx.x; i < tl; i += kOT) {
        sA[i] = cf[t0 + i];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          sB[j][i] = cf[2 * K + (int64_t)j * K + t0 + i];
          sC[j][i] = cf[2 * K + (int64_t)(D + j) * K + t0 + i];
        }
      }
      __syncthreads();
      for (int c0 = 0; c0 < tl; c0 += 8) {
        float a0[8], a1[8];
        float cm0 = -INFINITY, cm1 = -INFINITY;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int i = c0 + q;
          const bool in = i < tl;
          const int ii = in ? i : 0;
          float v0 = in ? sA[ii] : -INFINITY;
          float v1 = v0;
#pragma unroll
          for (int j = 0; j < D; ++j) {
            v0 = __builtin_fmaf(sB[j][ii], x0[j], v0);
            v0 = __builtin_fmaf(sC[j][ii], q0[j], v0);
            v1 = __builtin_fmaf(sB[j][ii], x1[j], v1);
            v1 = __builtin_fmaf(sC[j][ii], q1[j], v1);
          }
          a0[q] = v0;
          a1[q] = v1;
          cm0 = fmaxf(cm0, v0);
          cm1 = fmaxf(cm1, v1);
        }
        if (cm0 > m0) {
          s0 *= __builtin_amdgcn_exp2f(m0 - cm0);
          m0 = cm0;
        }
        if (cm1 > m1) {
          s1 *= __builtin_amdgcn_exp2f(m1 - cm1);
          m1 = cm1;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          s0 += __builtin_amdgcn_exp2f(a0[q] - m0);
          s1 += __builtin_amdgcn_exp2f(a1[q] - m1);
        }
      }
    }
    if (ok0) {
      if (!(m0 > -1e30f && s0 > 0.f && s0 < INFINITY)) bad |= FLAG_COL;
      const double l0 = ((double)m0 + (double)__builtin_amdgcn_logf(s0)) * kLn2;
      logD[n0] = l0;
      obj = __builtin_fma(h ? h[n0] : 1.0, l0, obj);
    }
    if (ok1) {
      if (!(m1 > -1e30f && s1 > 0.f && s1 < INFINITY)) bad |= FLAG_COL;
      const double l1 = ((double)m1 + (double)__builtin_amdgcn_logf(s1)) * kLn2;
      logD[n0 + 1] = l1;
      obj = __builtin_fma(h ? h[n0 + 1] : 1.0, l1, obj);
    }
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) obj += __shfl_xor(obj, off, 64);
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = obj;
  if (bad) atomicOr(&fl, bad);
  __syncthreads();
  if (threadIdx.x == 0) {
    double o = wred[0];
    for (int w = 1; w < kOT / 64; ++w) o += wred[w];
    part_obj[blockIdx.x] = o;
    part_flags[blockIdx.x] = fl;
  }
}

template <int D>
__global__ void __launch_bounds__(kOT)
    otf32_statepass_kernel(int K, int64_t N, const float* __restrict__ xf,
                           const float* __restrict__ cf, const double* __restrict__ h,
                           const double* __restrict__ logD, double* __restrict__ part) {
  constexpr int R = kOStates / 4;  // states per thread
  const int lc = threadIdx.x & 63;
  const int rg = threadIdx.x >> 6;
  const int kbase = blockIdx.y * kOStates + rg;
  float A[R], B[D][R], C[D][R], acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int k = kbase + 4 * r;
    const bool in = k < K;
    A[r] = in ? cf[K + k] : -INFINITY;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      B[j][r] = in ? cf[2 * K + (int64_t)j * K + k] : 0.f;
      C[j][r] = in ? cf[2 * K + (int64_t)(D + j) * K + k] : 0.f;
    }
    acc[r] = 0.f;
  }
  const int64_t stride = (int64_t)gridDim.x * 128;
  for (int64_t n0 = (int64_t)blockIdx.x * 128 + lc * 2; n0 < N; n0 += stride) {
    const bool two = n0 + 1 < N;
    float x0[D], x1[D], q0[D], q1[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      x0[j] = xf[n0 * D + j];
      x1[j] = two ? xf[(n0 + 1) * D + j] : x0[j];
      q0[j] = x0[j] * x0[j];
      q1[j] = x1[j] * x1[j];
    }
    const float e0 = (float)(-kLog2e * logD[n0]);
    // a missing second column contributes exp2(-inf) = 0
    const float e1 = two ? (float)(-kLog2e * logD[n0 + 1]) : -INFINITY;
    // bin multiplicities (exact in FP32 below 2^24 samples per bin)
    const float h0 = h ? (float)h[n0] : 1.f;
    const float h1 = h && two ? (float)h[n0 + 1] : 1.f;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      float v0 = A[r] + e0, v1 = A[r] + e1;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        v0 = __builtin_fmaf(B[j][r], x0[j], v0);
        v0 = __builtin_fmaf(C[j][r], q0[j], v0);
        v1 = __builtin_fmaf(B[j][r], x1[j], v1);
        v1 = __builtin_fmaf(C[j][r], q1[j], v1);
      }
      acc[r] = __builtin_fmaf(h0, __builtin_amdgcn_exp2f(v0), acc[r]);
      acc[r] = __builtin_fmaf(h1, __builtin_amdgcn_exp2f(v1), acc[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double v = (double)acc[r];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    const int k = kbase + 4 * r;
    if (lc == 0 && k < K) part[(int64_t)k * gridDim.x + blockIdx.x] = v;
  }
}

// ---- FP64 passes ----------------------------------------------------------------

// SPLIT: block (x, y) takes only the states [y kc, (y + 1) kc) and writes, per
// sample, the pair (max, sum) of its slice to pm[(y N + n) * 2] (the maximum
// is NaN for non-finite coordinates); otf64_colmerge_kernel combines them.
// This spreads columns with few samples over more workgroups.
template <int D, int MODEL, bool SPLIT>
__global__ void __launch_bounds__(kOT)
    otf64_colpass_kernel(int K, int64_t N, const double* __restrict__ xi,
                         const double* __restrict__ c64, const double* __restrict__ h,
                         double* __restrict__ logD,
                         double* __restrict__ part_obj, unsigned* __restrict__ part_flags,
                         int kc, double* __restrict__ pm) {
  constexpr int T = kOTile / 2;  // FP64 tile: half the states of the FP32 tile
  __shared__ double sE[T];
  __shared__ double sH[D][T];
  __shared__ double sX[D][T];
  __shared__ double wred[kOT / 64];
  __shared__ unsigned fl;
  if (threadIdx.x == 0) fl = 0u;
  double obj = 0.0;
  unsigned bad = 0;
  const int64_t stride = (int64_t)gridDim.x * kOT * 2;
  const int64_t n_iter = (N + stride - 1) / stride;
  for (int64_t it = 0; it < n_iter; ++it) {
    const int64_t n0 = it * stride + ((int64_t)blockIdx.x * kOT + threadIdx.x) * 2;
    const bool ok0 = n0 < N, ok1 = n0 + 1 < N;
    double x0[D], x1[D];
    double chk = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      x0[j] = ok0 ? xi[n0 * D + j] : 0.0;
      x1[j] = ok1 ? xi[(n0 + 1) * D + j] : x0[j];
      chk += x0[j] + x1[j];
    }
    if (chk != chk) bad |= FLAG_NAN;
    double m0 = -INFINITY, m1 = -INFINITY, s0 = 0.0, s1 = 0.0;
    const int kb = SPLIT ? min(K, (int)blockIdx.y * kc) : 0;
    const int ke = SPLIT ? min(K, kb + kc) : K;
    for (int t0 = kb; t0 < ke; t0 += T) {
      const int tl = min(T, ke - t0);
      __syncthreads();
      for (int i = threadIdx.x; i < tl; i += kOT) {
        sE[i] = c64[t0 + i];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          sH[j][i] = c64[2 * K + (int64_t)j * K + t0 + i];
          sX[j][i] = c64[2 * K + (int64_t)(D + j) * K + t0 + i];
        }
      }
      __syncthreads();
      for (int c0 = 0; c0 < tl; c0 += 8) {
        double a0[8], a1[8];
        double cm0 = -INFINITY, cm1 = -INFINITY;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int i = c0 + q;
          const bool in = i < tl;
          const int ii = in ? i : 0;
          double hc[D], xc[D];
#pragma unroll
          for (int j = 0; j < D; ++j) {
            hc[j] = sH[j][ii];
            xc[j] = sX[j][ii];
          }
          const double e = in ? sE[ii] : -INFINITY;
          a0[q] = e - model_rest<D, MODEL>(hc, xc, x0);
          a1[q] = e - model_rest<D, MODEL>(hc, xc, x1);
          cm0 = fmax(cm0, a0[q]);
          cm1 = fmax(cm1, a1[q]);
        }
        if (cm0 > m0) {
          s0 *= exp_nonpos(m0 - cm0);
          m0 = cm0;
        }
        if (cm1 > m1) {
          s1 *= exp_nonpos(m1 - cm1);
          m1 = cm1;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          s0 += exp_nonpos(a0[q] - m0);
          s1 += exp_nonpos(a1[q] - m1);
        }
      }
    }
    if constexpr (SPLIT) {
      const double nan_or = (chk != chk) ? NAN : 0.0;
      double* q = pm + ((int64_t)blockIdx.y * N + n0) * 2;
      if (ok0) {
        q[0] = m0 + nan_or;
        q[1] = s0;
      }
      if (ok1) {
        q[2] = m1 + nan_or;
        q[3] = s1;
      }
      continue;
    }
    if (ok0) {
      if (!(m0 > -INFINITY && m0 < INFINITY)) bad |= FLAG_COL;
      const double l0 = m0 + log(s0);
      logD[n0] = l0;
      obj = __builtin_fma(h ? h[n0] : 1.0, l0, obj);
    }
    if (ok1) {
      if (!(m1 > -INFINITY && m1 < INFINITY)) bad |= FLAG_COL;
      const double l1 = m1 + log(s1);
      logD[n0 + 1] = l1;
      obj = __builtin_fma(h ? h[n0 + 1] : 1.0, l1, obj);
    }
  }
  if constexpr (SPLIT) return;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) obj += __shfl_xor(obj, off, 64);
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = obj;
  if (bad) atomicOr(&fl, bad);
  __syncthreads();
  if (threadIdx.x == 0) {
    double o = wred[0];
    for (int w = 1; w < kOT / 64; ++w) o += wred[w];
    part_obj[blockIdx.x] = o;
    part_flags[blockIdx.x] = fl;
  }
}

// ln D_n from the Y slices of a split column pass: M = the largest slice
// maximum, S = sum over the slices (in order) of s_y exp(m_y - M); the
// objective partial and flags per block as in the column pass.
__global__ void __launch_bounds__(kOT)
    otf64_colmerge_kernel(int64_t N, int Y, const double* __restrict__ pm,
                          const double* __restrict__ h, double* __restrict__ logD,
                          double* __restrict__ part_obj, unsigned* __restrict__ part_flags) {
  __shared__ double wred[kOT / 64];
  __shared__ unsigned fl;
  if (threadIdx.x == 0) fl = 0u;
  __syncthreads();
  double obj = 0.0;
  unsigned bad = 0;
  for (int64_t n = (int64_t)blockIdx.x * kOT + threadIdx.x; n < N;
       n += (int64_t)gridDim.x * kOT) {
    double M = -INFINITY;
    bool nan = false;
    for (int y = 0; y < Y; ++y) {
      const double m = pm[((int64_t)y * N + n) * 2];
      nan = nan || (m != m);
      M = fmax(M, m);
    }
    double S = 0.0;
    if (M > -INFINITY && M < INFINITY)
      for (int y = 0; y < Y; ++y) {
        const double* q = pm + ((int64_t)y * N + n) * 2;
        S = __builtin_fma(q[1], exp_nonpos(q[0] - M), S);
      }
    if (nan) bad |= FLAG_NAN;
    if (!(M > -INFINITY && M < INFINITY)) bad |= FLAG_COL;
    const double l = M + log(S);
    logD[n] = l;
    obj = __builtin_fma(h ? h[n] : 1.0, l, obj);
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) obj += __shfl_xor(obj, off, 64);
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = obj;
  if (bad) atomicOr(&fl, bad);
  __syncthreads();
  if (threadIdx.x == 0) {
    double o = wred[0];
    for (int w = 1; w < kOT / 64; ++w) o += wred[w];
    part_obj[blockIdx.x] = o;
    part_flags[blockIdx.x] = fl;
  }
}

template <int D, int MODEL>
__global__ void __launch_bounds__(kOT)
    otf64_statepass_kernel(int K, int64_t N, const double* __restrict__ xi,
                           const double* __restrict__ c64, const double* __restrict__ h,
                           const double* __restrict__ logD, double* __restrict__ part) {
  constexpr int R = kOStates / 8;  // 8 states per thread; two row-group passes per block
  const int lc = threadIdx.x & 63;
  const int rg = threadIdx.x >> 6;
  const int64_t stride = (int64_t)gridDim.x * 128;
#pragma unroll 1
  for (int half = 0; half < 2; ++half) {
    const int kbase = blockIdx.y * kOStates + half * (kOStates / 2) + rg;
    double E[R], H[D][R], X[D][R], acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k = kbase + 4 * r;
      const bool in = k < K;
      E[r] = in ? c64[K + k] : -INFINITY;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        H[j][r] = in ? c64[2 * K + (int64_t)j * K + k] : 0.0;
        X[j][r] = in ? c64[2 * K + (int64_t)(D + j) * K + k] : 0.0;
      }
      acc[r] = 0.0;
    }
    for (int64_t n0 = (int64_t)blockIdx.x * 128 + lc * 2; n0 < N; n0 += stride) {
      const bool two = n0 + 1 < N;
      double x0[D], x1[D];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        x0[j] = xi[n0 * D + j];
        x1[j] = two ? xi[(n0 + 1) * D + j] : x0[j];
      }
      const double l0 = logD[n0];
      const double l1 = two ? logD[n0 + 1] : INFINITY;  // exp(-inf) = 0 for a missing column
      const double w0 = h ? h[n0] : 1.0;
      const double w1 = h && two ? h[n0 + 1] : 1.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double hc[D], xc[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          hc[j] = H[j][r];
          xc[j] = X[j][r];
        }
        acc[r] = __builtin_fma(w0, exp_nonpos(E[r] - l0 - model_rest<D, MODEL>(hc, xc, x0)),
                               acc[r]);
        acc[r] = __builtin_fma(w1, exp_nonpos(E[r] - l1 - model_rest<D, MODEL>(hc, xc, x1)),
                               acc[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double v = acc[r];
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
      const int k = kbase + 4 * r;
      if (lc == 0 && k < K) part[(int64_t)k * gridDim.x + blockIdx.x] = v;
    }
  }
}

// W_nk = exp(f_k - u_kn - ln D_n), N x K sample-major, FP64 model.
template <int D, int MODEL>
__global__ void otf64_weights_kernel(int K, int64_t N, const double* __restrict__ xi,
                                     const double* __restrict__ coef,
                                     const double* __restrict__ f,
                                     const double* __restrict__ logD, double* __restrict__ W) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)K * N) return;
  const int64_t n = e / K;
  const int k = (int)(e % K);
  const double* ck = coef + (int64_t)k * (1 + 2 * D);
  double h[D], xc[D], x[D];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    x[j] = xi[n * D + j];
    if (MODEL == BUMBAR_MODEL_HARMONIC) {
      h[j] = 0.5 * ck[1 + 2 * j];
      xc[j] = ck[2 + 2 * j];
    } else {
      h[j] = ck[1 + j];
      xc[j] = 0.0;
    }
  }
  W[e] = exp_nonpos(f[k] - ck[0] - model_rest<D, MODEL>(h, xc, x) - logD[n]);
}

// ---- launchers ------------------------------------------------------------------

size_t otf_coef_floats(int K, int d) { return (size_t)K * (2 + 2 * d); }

hipError_t launch_pack_coords(hipStream_t s, int64_t n, const double* xi, float* xf) {
  hipLaunchKernelGGL(pack_coords_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, xi,
                     xf);
  return hipGetLastError();
}

// ---- FP64 passes for windows on a product grid (2-D harmonic) ----------------
// State k = (i, j): u_k(x, y) = a_k + hx_i (x - cx_i)^2 + hy_j (y - cy_j)^2, so
// exp(c_k - u_kn) = exp(c_k - a_k) g_i(x_n) h_j(y_n). Per sample the column
// sum is the bilinear form g^T C h with C_ij = sum over the states of cell
// (i, j) of exp(c_k - a_k - cmax); per block the state sums are
// exp(E_k - cmax) M_ij with M = sum_n g(n) h(n)^T w_n. The factors are shifted
// per sample so that the largest of each is 1 (mx, my), and the shifts cancel
// in w_n = h_n exp(cmax - mx - my - ln D_n). Every exponential and product is
// FP64; the result differs from the direct passes by rounding only. A sample
// whose shifted column sum falls below 1e-280 (its states all far below the
// largest c_k - a_k) gets its ln D from the direct sum over the K states.

constexpr int kST = 256;  // threads of the product-grid kernels

__global__ void __launch_bounds__(256)
    sep_prep_kernel(int K, int Ix, int Jy, int JM, const double* __restrict__ coef,
                    const double* __restrict__ cst, const double* __restrict__ gk,
                    const int* __restrict__ cstart, const int* __restrict__ cstates,
                    double* __restrict__ C, double* __restrict__ cmax) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double m = -INFINITY;
  for (int k = tid; k < K; k += 256)
    if (gk[k] != 0.0) m = fmax(m, cst[k] - coef[(int64_t)k * 5]);
  red[tid] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double cm = red[0] == -INFINITY ? 0.0 : red[0];
  for (int e = tid; e < Ix * JM; e += 256) {
    const int i = e / JM, j = e % JM;
    double sum = 0.0;
    if (j < Jy) {
      const int c = i * Jy + j;
      for (int q = cstart[c]; q < cstart[c + 1]; ++q) {
        const int k = cstates[q];
        if (gk[k] != 0.0) sum += exp_nonpos(cst[k] - coef[(int64_t)k * 5] - cm);
      }
    }
    C[e] = sum;
  }
  if (tid == 0) cmax[0] = cm;
}

// ln D at (x, y) from the K states directly (the per-sweep FP64 coefficients
// of otf64_coef_kernel, d = 2): maximum, then the shifted sum.
__device__ double sep_direct_logD(int K, const double* __restrict__ c64, double x, double y) {
  double m = -INFINITY;
  for (int k = 0; k < K; ++k) {
    const double dx = x - c64[4 * K + k], dy = y - c64[5 * K + k];
    const double a = c64[k] - __builtin_fma(c64[3 * K + k] * dy, dy, c64[2 * K + k] * dx * dx);
    m = fmax(m, a);
  }
  if (!(m > -INFINITY)) return m;
  double s = 0.0;
  for (int k = 0; k < K; ++k) {
    const double dx = x - c64[4 * K + k], dy = y - c64[5 * K + k];
    const double a = c64[k] - __builtin_fma(c64[3 * K + k] * dy, dy, c64[2 * K + k] * dx * dx);
    s += exp_nonpos(a - m);
  }
  return m + log(s);
}

template <int JM>
__global__ void __launch_bounds__(kST)
    sep_colpass_kernel(int K, int64_t N, const double* __restrict__ xi,
                       const double* __restrict__ c64, int Ix, int Jy,
                       const double* __restrict__ fx, const double* __restrict__ fy,
                       const double* __restrict__ C, const double* __restrict__ cmax,
                       const double* __restrict__ h, double* __restrict__ logD,
                       double* __restrict__ part_obj, unsigned* __restrict__ part_flags) {
  __shared__ double wred[kST / 64];
  __shared__ unsigned fl;
  if (threadIdx.x == 0) fl = 0u;
  const double cm = cmax[0];
  double obj = 0.0;
  unsigned bad = 0;
  const int64_t stride = (int64_t)gridDim.x * kST;
  for (int64_t n = (int64_t)blockIdx.x * kST + threadIdx.x; n < N; n += stride) {
    const double x = xi[2 * n], y = xi[2 * n + 1];
    if ((x + y) != (x + y)) bad |= FLAG_NAN;
    // y factors, shifted so that the largest is 1 (padding: 0)
    double hv[JM];
    double my = INFINITY;
#pragma unroll
    for (int j = 0; j < JM; ++j) {
      const double dy = y - fy[2 * j + 1];
      const double q = j < Jy ? fy[2 * j] * dy * dy : INFINITY;
      hv[j] = q;
      my = fmin(my, q);
    }
#pragma unroll
    for (int j = 0; j < JM; ++j) hv[j] = exp_nonpos(my - hv[j]);
    double mx = INFINITY;
    for (int i = 0; i < Ix; ++i) {
      const double dx = x - fx[2 * i + 1];
      mx = fmin(mx, fx[2 * i] * dx * dx);
    }
    double Dp = 0.0;
    for (int i = 0; i < Ix; ++i) {
      const double dx = x - fx[2 * i + 1];
      const double g = exp_nonpos(mx - fx[2 * i] * dx * dx);
      const double* Ci = C + (int64_t)i * JM;
      double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll
      for (int j = 0; j < JM; j += 4) {
        t0 = __builtin_fma(Ci[j], hv[j], t0);
        t1 = __builtin_fma(Ci[j + 1], hv[j + 1], t1);
        t2 = __builtin_fma(Ci[j + 2], hv[j + 2], t2);
        t3 = __builtin_fma(Ci[j + 3], hv[j + 3], t3);
      }
      Dp = __builtin_fma(g, (t0 + t1) + (t2 + t3), Dp);
    }
    const double l = Dp >= 1e-280 ? cm - mx - my + log(Dp) : sep_direct_logD(K, c64, x, y);
    if (!(l > -INFINITY && l < INFINITY)) bad |= FLAG_COL;
    logD[n] = l;
    obj = __builtin_fma(h ? h[n] : 1.0, l, obj);
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) obj += __shfl_xor(obj, off, 64);
  if ((threadIdx.x & 63) == 0) wred[threadIdx.x >> 6] = obj;
  if (bad) atomicOr(&fl, bad);
  __syncthreads();
  if (threadIdx.x == 0) {
    double o = wred[0];
    for (int w = 1; w < kST / 64; ++w) o += wred[w];
    part_obj[blockIdx.x] = o;
    part_flags[blockIdx.x] = fl;
  }
}

// State pass: chunks of 32 samples; eight threads per sample fill the shifted
// factors (g, and h times w_n) into LDS, then thread (ti, tj) of 16 x 16
// accumulates M_ij for i = ti + 16 a (a < IA) and j = tj + 16 b (b < JB).
template <int IA, int JB>
__global__ void __launch_bounds__(kST)
    sep_statepass_kernel(int K, int64_t N, const double* __restrict__ xi,
                         const double* __restrict__ c64, int Ix, int Jy,
                         const double* __restrict__ fx, const double* __restrict__ fy,
                         const int* __restrict__ ix, const int* __restrict__ jy,
                         const double* __restrict__ cmax, const double* __restrict__ h,
                         const double* __restrict__ logD, double* __restrict__ part) {
  constexpr int NS = 32;            // samples per chunk
  constexpr int RP = kSepMax + 1;   // padded LDS row
  __shared__ double buf[2 * NS * RP];
  double(*Gs)[RP] = reinterpret_cast<double(*)[RP]>(buf);
  double(*Hs)[RP] = reinterpret_cast<double(*)[RP]>(buf + NS * RP);
  const int tid = threadIdx.x;
  const int ti = tid & 15, tj = tid >> 4;
  const int sl = tid >> 3, r = tid & 7;  // sample of the chunk, and its eighth of the factors
  const double cm = cmax[0];
  double acc[IA][JB];
#pragma unroll
  for (int a = 0; a < IA; ++a)
#pragma unroll
    for (int b = 0; b < JB; ++b) acc[a][b] = 0.0;
  const int64_t nchunks = (N + NS - 1) / NS;
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int64_t n = c * NS + sl;
    const bool in = n < N;
    const double x = in ? xi[2 * n] : 0.0, y = in ? xi[2 * n + 1] : 0.0;
    double mx = INFINITY, my = INFINITY;
    for (int i = r; i < Ix; i += 8) {
      const double dx = x - fx[2 * i + 1];
      mx = fmin(mx, fx[2 * i] * dx * dx);
    }
    for (int j = r; j < Jy; j += 8) {
      const double dy = y - fy[2 * j + 1];
      my = fmin(my, fy[2 * j] * dy * dy);
    }
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
      mx = fmin(mx, __shfl_xor(mx, off, 64));
      my = fmin(my, __shfl_xor(my, off, 64));
    }
    const double w = in ? (h ? h[n] : 1.0) * exp(cm - mx - my - logD[n]) : 0.0;
    __syncthreads();  // the previous chunk's products are done
    for (int i = r; i < 16 * IA; i += 8) {
      double g = 0.0;
      if (i < Ix) {
        const double dx = x - fx[2 * i + 1];
        g = exp_nonpos(mx - fx[2 * i] * dx * dx);
      }
      Gs[sl][i] = g;
    }
    for (int j = r; j < 16 * JB; j += 8) {
      double v = 0.0;
      if (j < Jy) {
        const double dy = y - fy[2 * j + 1];
        v = w * exp_nonpos(my - fy[2 * j] * dy * dy);
      }
      Hs[sl][j] = v;
    }
    __syncthreads();
    for (int t = 0; t < NS; ++t) {
      double ga[IA], hb[JB];
#pragma unroll
      for (int a = 0; a < IA; ++a) ga[a] = Gs[t][ti + 16 * a];
#pragma unroll
      for (int b = 0; b < JB; ++b) hb[b] = Hs[t][tj + 16 * b];
#pragma unroll
      for (int a = 0; a < IA; ++a)
#pragma unroll
        for (int b = 0; b < JB; ++b) acc[a][b] = __builtin_fma(ga[a], hb[b], acc[a][b]);
    }
  }
  // M in LDS (64 x 65 fits in buf), then the per-state partials
  double(*Ms)[RP] = reinterpret_cast<double(*)[RP]>(buf);
  __syncthreads();
#pragma unroll
  for (int a = 0; a < IA; ++a)
#pragma unroll
    for (int b = 0; b < JB; ++b) Ms[ti + 16 * a][tj + 16 * b] = acc[a][b];
  __syncthreads();
  for (int k = tid; k < K; k += kST) {
    const double M = Ms[ix[k]][jy[k]];
    const double z = c64[K + k] - cm;
    double v = 0.0;
    if (M > 0.0) v = z < 600.0 ? exp(z) * M : exp(z + log(M));
    part[(int64_t)k * gridDim.x + blockIdx.x] = v;
  }
}

size_t sep_int_count(int K) { return 3 * (size_t)K + (size_t)kSepMax * kSepMax + 1; }
size_t sep_double_count() { return 4 * (size_t)kSepMax + (size_t)kSepMax * kSepMax + 8; }

static hipError_t launch_sweep_sep(hipStream_t s, const OtfModel& m, int K, int64_t N,
                                   const double* cst, const double* gk, const double* h,
                                   double* logD, double* part, double* part_obj,
                                   unsigned* part_flags, int G) {
  const SepGrid& g = *m.sep;
  hipLaunchKernelGGL(sep_prep_kernel, dim3(1), dim3(256), 0, s, K, g.Ix, g.Jy, g.JM, m.coef, cst,
                     gk, g.cstart, g.cstates, g.C, g.cmax);
#define SEP_COL(JM_)                                                                              \
  case JM_:                                                                                       \
    hipLaunchKernelGGL(sep_colpass_kernel<JM_>, dim3(G), dim3(kST), 0, s, K, N, m.xi, m.cf64,      \
                       g.Ix, g.Jy, g.fx, g.fy, g.C, g.cmax, h, logD, part_obj, part_flags);       \
    break;
  switch (g.JM) {
    SEP_COL(8) SEP_COL(16) SEP_COL(24) SEP_COL(32) SEP_COL(40) SEP_COL(48) SEP_COL(56) SEP_COL(64)
    default:
      return hipErrorInvalidValue;
  }
#undef SEP_COL
#define SEP_STATE(IA_, JB_)                                                                       \
  case 4 * (IA_ - 1) + JB_ - 1:                                                                   \
    hipLaunchKernelGGL((sep_statepass_kernel<IA_, JB_>), dim3(G), dim3(kST), 0, s, K, N, m.xi,     \
                       m.cf64, g.Ix, g.Jy, g.fx, g.fy, g.ix, g.jy, g.cmax, h, logD, part);        \
    break;
  // 16-row groups of the x and y factors (Ix, Jy <= 64)
  switch (4 * ((g.Ix + 15) / 16 - 1) + (g.Jy + 15) / 16 - 1) {
    SEP_STATE(1, 1) SEP_STATE(1, 2) SEP_STATE(1, 3) SEP_STATE(1, 4)
    SEP_STATE(2, 1) SEP_STATE(2, 2) SEP_STATE(2, 3) SEP_STATE(2, 4)
    SEP_STATE(3, 1) SEP_STATE(3, 2) SEP_STATE(3, 3) SEP_STATE(3, 4)
    SEP_STATE(4, 1) SEP_STATE(4, 2) SEP_STATE(4, 3) SEP_STATE(4, 4)
    default:
      return hipErrorInvalidValue;
  }
#undef SEP_STATE
  return hipGetLastError();
}

hipError_t launch_otf_coefs(hipStream_t s, const OtfModel& m, bool fp32, int K, const double* cst,
                            const double* gk) {
  const dim3 cg((K + 255) / 256);
  if (fp32)
    hipLaunchKernelGGL(otf32_coef_kernel, cg, dim3(256), 0, s, K, m.d, m.model, m.coef, cst, gk,
                       m.cf32);
  else
    hipLaunchKernelGGL(otf64_coef_kernel, cg, dim3(256), 0, s, K, m.d, m.model, m.coef, cst, gk,
                       m.cf64);
  return hipGetLastError();
}

hipError_t launch_sweep_otf(hipStream_t s, const OtfModel& m, bool fp32, int K, int64_t N,
                            const double* cst, const double* gk, const double* h, double* logD,
                            double* part, size_t part_cap,
                            double* part_obj, unsigned* part_flags, int num_cus, int* grid_out) {
  if (m.d != 1 && m.d != 2) return hipErrorInvalidValue;
  const int G = otf_grid(N, num_cus);
  *grid_out = G;
  const dim3 sg(G, (K + kOStates - 1) / kOStates);
  hipError_t e = launch_otf_coefs(s, m, fp32, K, cst, gk);
  if (e != hipSuccess) return e;
  if (!fp32 && m.sep && m.d == 2 && m.model == BUMBAR_MODEL_HARMONIC) {
    // a workgroup per 64 samples (two state-pass chunks), up to the partial
    // buffers' capacity: a workgroup's chunks run one after another, each a
    // chain of dependent loads and FP64 exponentials, so on a binned level
    // the pass takes as long as one workgroup's share (512 samples per
    // workgroup cost about 90 us whatever the level size)
    int64_t gs = (N + 63) / 64;
    if (gs > sweep_max_grid(num_cus)) gs = sweep_max_grid(num_cus);
    *grid_out = (int)gs;
    return launch_sweep_sep(s, m, K, N, cst, gk, h, logD, part, part_obj, part_flags, (int)gs);
  }
  if (fp32) {
    if (m.d == 1) {
      hipLaunchKernelGGL(otf32_colpass_kernel<1>, dim3(G), dim3(kOT), 0, s, K, N, m.xf, m.cf32,
                         h, logD, part_obj, part_flags);
      hipLaunchKernelGGL(otf32_statepass_kernel<1>, sg, dim3(kOT), 0, s, K, N, m.xf, m.cf32, h,
                         logD, part);
    } else {
      hipLaunchKernelGGL(otf32_colpass_kernel<2>, dim3(G), dim3(kOT), 0, s, K, N, m.xf, m.cf32,
                         h, logD, part_obj, part_flags);
      hipLaunchKernelGGL(otf32_statepass_kernel<2>, sg, dim3(kOT), 0, s, K, N, m.xf, m.cf32, h,
                         logD, part);
    }
    return hipGetLastError();
  }
  // few column blocks: the states split over Y slices (pairs in part, then merged)
  int Y = 1;
  if (G < num_cus) {
    Y = std::min((K + 63) / 64, (2 * num_cus + G - 1) / G);
    while (Y > 1 && (size_t)Y * (size_t)N * 2 > part_cap) --Y;
  }
  const int kc = (K + Y - 1) / Y;
#define OTF64_PASSES(D_, M_)                                                                      \
  if (Y > 1) {                                                                                    \
    hipLaunchKernelGGL((otf64_colpass_kernel<D_, M_, true>), dim3(G, Y), dim3(kOT), 0, s, K, N,   \
                       m.xi, m.cf64, h, logD, part_obj, part_flags, kc, part);                     \
    hipLaunchKernelGGL(otf64_colmerge_kernel, dim3(G), dim3(kOT), 0, s, N, Y, part, h, logD,      \
                       part_obj, part_flags);                                                     \
  } else {                                                                                        \
    hipLaunchKernelGGL((otf64_colpass_kernel<D_, M_, false>), dim3(G), dim3(kOT), 0, s, K, N,     \
                       m.xi, m.cf64, h, logD, part_obj, part_flags, kc, nullptr);                  \
  }                                                                                               \
  hipLaunchKernelGGL((otf64_statepass_kernel<D_, M_>), sg, dim3(kOT), 0, s, K, N, m.xi, m.cf64,   \
                     h, logD, part)
  if (m.model == BUMBAR_MODEL_HARMONIC) {
    if (m.d == 1) {
      OTF64_PASSES(1, BUMBAR_MODEL_HARMONIC);
    } else {
      OTF64_PASSES(2, BUMBAR_MODEL_HARMONIC);
    }
  } else {
    if (m.d == 1) {
      OTF64_PASSES(1, BUMBAR_MODEL_LINEAR);
    } else {
      OTF64_PASSES(2, BUMBAR_MODEL_LINEAR);
    }
  }
#undef OTF64_PASSES
  return hipGetLastError();
}

hipError_t launch_weights_otf(hipStream_t s, const OtfModel& m, int K, int64_t N, const double* f,
                              const double* logD, double* W) {
  const int64_t tot = (int64_t)K * N;
  const dim3 g((unsigned)((tot + 255) / 256));
  if (m.model == BUMBAR_MODEL_HARMONIC) {
    if (m.d == 1)
      hipLaunchKernelGGL((otf64_weights_kernel<1, BUMBAR_MODEL_HARMONIC>), g, dim3(256), 0, s, K,
                         N, m.xi, m.coef, f, logD, W);
    else
      hipLaunchKernelGGL((otf64_weights_kernel<2, BUMBAR_MODEL_HARMONIC>), g, dim3(256), 0, s, K,
                         N, m.xi, m.coef, f, logD, W);
  } else {
    if (m.d == 1)
      hipLaunchKernelGGL((otf64_weights_kernel<1, BUMBAR_MODEL_LINEAR>), g, dim3(256), 0, s, K, N,
                         m.xi, m.coef, f, logD, W);
    else
      hipLaunchKernelGGL((otf64_weights_kernel<2, BUMBAR_MODEL_LINEAR>), g, dim3(256), 0, s, K, N,
                         m.xi, m.coef, f, logD, W);
  }
  return hipGetLastError();
}

}  // namespace bumbar
