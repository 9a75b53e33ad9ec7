// Unbinned / binned sweep for many states (K beyond the register-tiled
// single-pass kernel): two passes over u, FP64 arithmetic, u in FP64 or FP32.
//
// Pass A (column pass): for each column n the exact log-sum-exp over the
// sampled states, ln D_n = LSE_k(c_k - u_kn), as a running (max, sum) pair
// updated in chunks of 8 states (one extra exponential per chunk when the
// running maximum moves), plus the objective partial sum_n h_n ln D_n and a
// NaN check.
// Pass B (state pass): acc_k += h_n exp(c_k - u_kn - ln D_n) with the states
// split into blocks of 64 (grid.y) so each thread keeps 16 accumulators; the
// samples are split over grid.x persistent blocks whose partials are written
// state-major for the finaliser (the same layout as the single-pass kernel).
// u is read twice; each element costs about 2.1 exponentials.
#include <cmath>

#include "bumbar_impl.h"
#include "devmath.h"

namespace bumbar {

constexpr int kWA = 256;     // pass A threads (2 columns each)
constexpr int kWB = 256;     // pass B threads: 4 row groups x 64 lanes
constexpr int kWBStates = 64;  // states per pass-B block
constexpr int kWBRows = kWBStates / 4;

int wide_grid(int64_t N, int num_cus) {
  int64_t g = (N + 2 * kWA - 1) / (2 * kWA);
  const int64_t cap = (int64_t)num_cus * 4;
  if (g > cap) g = cap;
  if (g > sweep_max_grid(num_cus)) g = sweep_max_grid(num_cus);
  return (int)(g < 1 ? 1 : g);
}

template <typename TI>
__global__ void __launch_bounds__(kWA)
    wide_colpass_kernel(const TI* __restrict__ u, int64_t ld, int K, int64_t N,
                        const double* __restrict__ cst, const double* __restrict__ gk,
                        const double* __restrict__ h, double* __restrict__ logD,
                        double* __restrict__ part_obj, unsigned* __restrict__ part_flags) {
  extern __shared__ double csd[];  // K values: c_k for sampled states, -inf otherwise
  __shared__ double wred[kWA / 64];
  __shared__ unsigned fl;
  for (int k = threadIdx.x; k < K; k += kWA) csd[k] = gk[k] != 0.0 ? cst[k] : -INFINITY;
  if (threadIdx.x == 0) fl = 0u;
  __syncthreads();
  double obj = 0.0;
  unsigned bad = 0;
  const int64_t stride = (int64_t)gridDim.x * kWA * 2;
  for (int64_t n0 = ((int64_t)blockIdx.x * kWA + threadIdx.x) * 2; n0 < N; n0 += stride) {
    const bool two = n0 + 1 < N;
    double m0 = -INFINITY, m1 = -INFINITY, s0 = 0.0, s1 = 0.0, chk = 0.0;
    const TI* p = u + n0;
    for (int k0 = 0; k0 < K; k0 += 8) {
      double a0[8], a1[8];
      double cm0 = -INFINITY, cm1 = -INFINITY;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = k0 + q;
        const bool ok = k < K;
        const TI* pk = p + (int64_t)(ok ? k : 0) * ld;
        const double x0 = (double)pk[0];
        const double x1 = two ? (double)pk[1] : x0;
        const double c = ok ? csd[k] : -INFINITY;
        a0[q] = c - x0;
        a1[q] = c - x1;
        chk += ok ? x0 + x1 : 0.0;
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
    if (chk != chk) bad |= FLAG_NAN;
    if (!(m0 > -INFINITY && m0 < INFINITY)) bad |= FLAG_COL;
    const double l0 = m0 + log(s0);
    logD[n0] = l0;
    obj = __builtin_fma(h ? h[n0] : 1.0, l0, obj);
    if (two) {
      if (!(m1 > -INFINITY && m1 < INFINITY)) bad |= FLAG_COL;
      const double l1 = m1 + log(s1);
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
    for (int w = 1; w < kWA / 64; ++w) o += wred[w];
    part_obj[blockIdx.x] = o;
    part_flags[blockIdx.x] = fl;
  }
}

template <typename TI>
__global__ void __launch_bounds__(kWB)
    wide_statepass_kernel(const TI* __restrict__ u, int64_t ld, int K, int64_t N,
                          const double* __restrict__ cst, const double* __restrict__ h,
                          const double* __restrict__ logD, double* __restrict__ part) {
  const int lc = threadIdx.x & 63;
  const int rg = threadIdx.x >> 6;
  const int kbase = blockIdx.y * kWBStates + rg;
  double c[kWBRows], acc[kWBRows];
#pragma unroll
  for (int j = 0; j < kWBRows; ++j) {
    const int k = kbase + 4 * j;
    c[j] = k < K ? cst[k] : -INFINITY;
    acc[j] = 0.0;
  }
  const int64_t stride = (int64_t)gridDim.x * 128;
  for (int64_t n0 = (int64_t)blockIdx.x * 128 + lc * 2; n0 < N; n0 += stride) {
    const bool two = n0 + 1 < N;
    const double l0 = logD[n0];
    const double l1 = two ? logD[n0 + 1] : 0.0;
    const double h0 = h ? h[n0] : 1.0;
    const double h1 = two ? (h ? h[n0 + 1] : 1.0) : 0.0;
#pragma unroll
    for (int j = 0; j < kWBRows; ++j) {
      const int k = kbase + 4 * j;
      const TI* pk = u + (int64_t)(k < K ? k : 0) * ld + n0;
      const double x0 = (double)pk[0];
      const double x1 = two ? (double)pk[1] : x0;
      acc[j] = __builtin_fma(h0, exp_nonpos(c[j] - x0 - l0), acc[j]);
      acc[j] = __builtin_fma(h1, exp_nonpos(c[j] - x1 - l1), acc[j]);
    }
  }
  // reduce over the 64 lanes of each row group (one wave), write state-major
#pragma unroll
  for (int j = 0; j < kWBRows; ++j) {
    double v = acc[j];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    const int k = kbase + 4 * j;
    if (lc == 0 && k < K) part[(int64_t)k * gridDim.x + blockIdx.x] = v;
  }
}

template <typename TI>
static hipError_t launch_wide_t(hipStream_t s, const TI* u, int64_t ld, int K, int64_t N,
                                const double* cst, const double* gk, const double* h,
                                double* logD, double* part, double* part_obj,
                                unsigned* part_flags, int num_cus, int* grid_out) {
  const int G = wide_grid(N, num_cus);
  *grid_out = G;
  const size_t lds = sizeof(double) * (size_t)K;
  // allow up to 144 KB of dynamic LDS (K <= 18432 states) once
  static const bool attr = [] {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&wide_colpass_kernel<TI>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 144 * 1024) != hipSuccess)
      (void)hipGetLastError();
    return true;
  }();
  (void)attr;
  if (lds > 144 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(wide_colpass_kernel<TI>, dim3(G), dim3(kWA), lds, s, u, ld, K, N, cst, gk, h,
                     logD, part_obj, part_flags);
  dim3 gb(G, (K + kWBStates - 1) / kWBStates);
  hipLaunchKernelGGL(wide_statepass_kernel<TI>, gb, dim3(kWB), 0, s, u, ld, K, N, cst, h, logD,
                     part);
  return hipGetLastError();
}

hipError_t launch_sweep_wide(hipStream_t s, const void* u, bool f32, int64_t ld, int K, int64_t N,
                             const double* cst, const double* gk, const double* h, double* logD,
                             double* part, double* part_obj, unsigned* part_flags, int num_cus,
                             int* grid_out) {
  if (f32)
    return launch_wide_t<float>(s, reinterpret_cast<const float*>(u), ld, K, N, cst, gk, h, logD,
                                part, part_obj, part_flags, num_cus, grid_out);
  return launch_wide_t<double>(s, reinterpret_cast<const double*>(u), ld, K, N, cst, gk, h, logD,
                               part, part_obj, part_flags, num_cus, grid_out);
}

}  // namespace bumbar
