// Mixed-precision sweep: u_kn packed to FP32 with per-column and per-state
// shifts, FP32 arithmetic inside a tile, FP64 for everything that
// accumulates across tiles and iterations.
//
// Packing at a reference point f0 (c0_k = ln N'_k + f0_k):
//   m0_n = max_k (c0_k - u_kn)            (FP64, kept per column)
//   r_kn = fp32(c0_k - u_kn - m0_n) <= 0  (FP32, K x N)
// so the entries that carry weight sit near 0, where FP32 keeps ~7 digits of
// the exponent. At a later f the sweep needs a_kn = c_k - u_kn - m0_n =
// r_kn + d_k with d_k = f_k - f0_k (small): the kernel below is the FP64
// single-pass kernel with T = float, a = d_k + r, e = 2^((a - m) log2 e) on
// the hardware exponential, column sums and per-thread state accumulators in
// FP32, the per-workgroup partials written in FP64 and merged by the FP64
// finaliser (ln D_n = m0_n + m_n + ln D'_n in FP64).
#include <cmath>

#include "bumbar_impl.h"
#include "devmath.h"

namespace bumbar {

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float exp_f32(float x) {
  // v_exp_f32 computes 2^x; exp(x) = 2^(x log2 e). Arguments are <= 0 here;
  // -inf gives 0.
  return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
}

// Pack: one thread per column, two passes over the column (the second from
// cache). Rows past K do not exist here; unsampled states take part in the
// maximum so every r <= 0.
// u is FP64, or FP32 (widened: the differences are taken in FP64 either way).
template <typename TI>
__global__ void __launch_bounds__(256)
    pack_f32_kernel(const TI* __restrict__ u, int64_t ld, int K, int64_t N,
                    const double* __restrict__ c0, float* __restrict__ r, int64_t ldr,
                    double* __restrict__ m0) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  double m = -INFINITY;
  for (int k = 0; k < K; ++k) m = fmax(m, c0[k] - (double)u[(int64_t)k * ld + n]);
  if (!(m > -INFINITY && m < INFINITY)) m = 0.0;
  m0[n] = m;
  for (int k = 0; k < K; ++k)
    r[(int64_t)k * ldr + n] = (float)(c0[k] - (double)u[(int64_t)k * ld + n] - m);
}

hipError_t launch_pack_f32(hipStream_t s, const void* u, bool f32, int64_t ld, int K, int64_t N,
                           const double* c0, float* r, int64_t ldr, double* m0) {
  const dim3 grid((unsigned)((N + 255) / 256));
  if (f32)
    hipLaunchKernelGGL(pack_f32_kernel<float>, grid, dim3(256), 0, s,
                       reinterpret_cast<const float*>(u), ld, K, N, c0, r, ldr, m0);
  else
    hipLaunchKernelGGL(pack_f32_kernel<double>, grid, dim3(256), 0, s,
                       reinterpret_cast<const double*>(u), ld, K, N, c0, r, ldr, m0);
  return hipGetLastError();
}

// d_k = f_k - f0_k (FP64 -> the kernel rounds once to FP32)
__global__ void delta_kernel(int K, const double* f, const double* f0, double* d) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) d[k] = f[k] - f0[k];
}

hipError_t launch_delta(hipStream_t s, int K, const double* f, const double* f0, double* d) {
  hipLaunchKernelGGL(delta_kernel, dim3((K + 255) / 256), dim3(256), 0, s, K, f, f0, d);
  return hipGetLastError();
}

// Single-pass FP32 sweep. Thread (lc, rg) owns rows rg + RG j and 4
// consecutive columns (16-byte loads) of each 64-column tile.
template <int NW, int ROWS>
__global__ void __launch_bounds__(NW * 64)
    sweep32_kernel(const float* __restrict__ r, int64_t ld, int K, int64_t N, int64_t ntiles,
                   const double* __restrict__ dk, const double* __restrict__ gk,
                   const double* __restrict__ m0, double* __restrict__ logD,
                   double* __restrict__ part, double* __restrict__ part_obj,
                   unsigned* __restrict__ part_flags) {
  constexpr int LPR = 16, CPL = 4, TN = LPR * CPL;
  constexpr int NT = NW * 64;
  constexpr int RG = NT / LPR;
  // two copies of the reduction buffers, alternating by tile: every wave reads
  // all of them in the ln D step, and a wave may reach the next tile's pass 1
  // before another has finished that step
  __shared__ float red1b[2][NW][TN];
  __shared__ float red2b[2][NW][TN];
  __shared__ float d_sh[ROWS * RG];
  __shared__ double wred[NW];
  __shared__ unsigned fl;
  const int tid = threadIdx.x;
  const int lc = tid % LPR;
  const int rg = tid / LPR;
  const int wave = tid >> 6;
  const int rgw = (tid & 63) / LPR;
  for (int k = tid; k < ROWS * RG; k += NT) d_sh[k] = (k < K) ? (float)dk[k] : -INFINITY;
  if (tid == 0) fl = 0u;
  unsigned smask = 0u;
  float acc[ROWS];
#pragma unroll
  for (int j = 0; j < ROWS; ++j) {
    const int k = rg + RG * j;
    if (k < K && gk[k] != 0.0) smask |= 1u << j;
    acc[j] = 0.0f;
  }
  const int rows_here = (rg < K) ? (K - 1 - rg) / RG + 1 : 0;
  const float* base = r + (int64_t)((rg < K) ? rg : 0) * ld + (int64_t)lc * CPL;
  const int64_t rstride = (int64_t)RG * ld;
  const unsigned valid_bits = (rows_here >= 32) ? 0xffffffffu : ((1u << rows_here) - 1u);
  const bool masked = __syncthreads_or(smask != valid_bits) != 0;
  const bool vec = ((reinterpret_cast<uintptr_t>(r) & 15) == 0) && ((ld & 3) == 0);
  double obj = 0.0;
  unsigned bad = 0;
  int par = 0;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x, par ^= 1) {
    float(*red1)[TN] = red1b[par];
    float(*red2)[TN] = red2b[par];
    const int64_t col0 = t * TN + (int64_t)lc * CPL;
    const bool full = (t + 1) * TN <= N;
    float a[ROWS][CPL];
    int rgo = rg;
    asm volatile("" : "+v"(rgo));
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      int64_t roff = (int64_t)(j < rows_here ? j : (rows_here > 0 ? rows_here - 1 : 0)) * rstride;
      asm volatile("" : "+v"(roff));
      const float* p = base + roff + t * TN;
      if (full && vec) {
        // the packed matrix is streamed once per sweep: non-temporal loads
        const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
        a[j][0] = v.x;
        a[j][1] = v.y;
        a[j][2] = v.z;
        a[j][3] = v.w;
      } else {
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
          const int64_t off = (col0 + i < N) ? (int64_t)i : (N - 1 - col0);
          a[j][i] = p[off];
        }
      }
    }
    float cm[CPL], chk = 0.0f;
#pragma unroll
    for (int i = 0; i < CPL; ++i) cm[i] = -INFINITY;
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      const float d = d_sh[rgo + RG * j];
#pragma unroll
      for (int i = 0; i < CPL; ++i) {
        a[j][i] = d + a[j][i];
        cm[i] = fmaxf(cm[i], a[j][i]);
        chk += a[j][i];
      }
    }
    if (chk != chk) bad |= FLAG_NAN;
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
#pragma unroll
      for (int off = LPR; off < 64; off <<= 1) cm[i] = fmaxf(cm[i], __shfl_xor(cm[i], off, 64));
      if (rgw == 0) red1[wave][lc * CPL + i] = cm[i];
    }
    __syncthreads();
    float m[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      float v = red1[0][lc * CPL + i];
#pragma unroll
      for (int w = 1; w < NW; ++w) v = fmaxf(v, red1[w][lc * CPL + i]);
      m[i] = (v == -INFINITY) ? 0.0f : v;
    }
    float ds[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) ds[i] = 0.0f;
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
      const bool g = !masked || ((smask >> j) & 1u);
#pragma unroll
      for (int i = 0; i < CPL; ++i) {
        a[j][i] = exp_f32(a[j][i] - m[i]);
        ds[i] += g ? a[j][i] : 0.0f;
      }
    }
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
#pragma unroll
      for (int off = LPR; off < 64; off <<= 1) ds[i] += __shfl_xor(ds[i], off, 64);
      if (rgw == 0) red2[wave][lc * CPL + i] = ds[i];
    }
    __syncthreads();
    float w[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      float D = red2[0][lc * CPL + i];
#pragma unroll
      for (int wv = 1; wv < NW; ++wv) D += red2[wv][lc * CPL + i];
      const bool valid = col0 + i < N;
      w[i] = valid ? 1.0f / D : 0.0f;
      if (valid && !(D >= 1e-30f && D <= 1e30f)) bad |= FLAG_COL;
    }
#pragma unroll
    for (int j = 0; j < ROWS; ++j)
#pragma unroll
      for (int i = 0; i < CPL; ++i) acc[j] = __builtin_fmaf(a[j][i], w[i], acc[j]);
    // ln D_n = m0_n + m_n + ln D'_n (FP64), one lane per column, spread over waves
    constexpr int CW = TN / NW;
    const int lane = tid & 63;
    if (lane < CW) {
      const int col = wave * CW + lane;
      float mv = red1[0][col], Dv = red2[0][col];
#pragma unroll
      for (int wv = 1; wv < NW; ++wv) {
        mv = fmaxf(mv, red1[wv][col]);
        Dv += red2[wv][col];
      }
      if (mv == -INFINITY) mv = 0.0f;
      const int64_t n = t * TN + col;
      if (n < N) {
        const double l = m0[n] + (double)mv + log_ge1((double)Dv);
        if (logD != nullptr) logD[n] = l;
        obj += l;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < ROWS; ++j) {
    double v = (double)acc[j];
#pragma unroll
    for (int off = 1; off < LPR; off <<= 1) v += __shfl_xor(v, off, 64);
    const int k = rg + RG * j;
    if (lc == 0 && k < K) part[(int64_t)k * gridDim.x + blockIdx.x] = v;
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) obj += __shfl_xor(obj, off, 64);
  if ((tid & 63) == 0) wred[wave] = obj;
  if (bad) atomicOr(&fl, bad);
  __syncthreads();
  if (tid == 0) {
    double o = wred[0];
    for (int wv = 1; wv < NW; ++wv) o += wred[wv];
    part_obj[blockIdx.x] = o;
    part_flags[blockIdx.x] = fl;
  }
}

struct Cfg32 {
  int kmax, nw, rows;
};
static const Cfg32 kCfg32[] = {{64, 4, 4}, {128, 4, 8}, {256, 4, 16}, {512, 8, 16}, {1024, 16, 16}};

bool sweep32_supported(int K) { return K <= 1024; }

template <int NW, int ROWS>
static hipError_t launch32_t(hipStream_t s, const float* r, int64_t ld, int K, int64_t N,
                             const double* dk, const double* gk, const double* m0, double* logD,
                             double* part, double* part_obj, unsigned* pf, int num_cus,
                             int* grid_out) {
  const int64_t ntiles = (N + 63) / 64;
  static const int per_cu = [] {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sweep32_kernel<NW, ROWS>, NW * 64, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    return nb;
  }();
  int64_t g = (int64_t)num_cus * per_cu;
  if (g > ntiles) g = ntiles;
  if (g > sweep_max_grid(num_cus)) g = sweep_max_grid(num_cus);
  if (g < 1) g = 1;
  *grid_out = (int)g;
  hipLaunchKernelGGL((sweep32_kernel<NW, ROWS>), dim3((unsigned)g), dim3(NW * 64), 0, s, r, ld, K,
                     N, ntiles, dk, gk, m0, logD, part, part_obj, pf);
  return hipGetLastError();
}

hipError_t launch_sweep32(hipStream_t s, const float* r, int64_t ld, int K, int64_t N,
                          const double* dk, const double* gk, const double* m0, double* logD,
                          double* part, double* part_obj, unsigned* part_flags, int num_cus,
                          int* grid_out) {
  for (const auto& c : kCfg32) {
    if (K > c.kmax) continue;
#define B32(a, b)                                                                               \
  if (c.nw == a && c.rows == b)                                                                 \
    return launch32_t<a, b>(s, r, ld, K, N, dk, gk, m0, logD, part, part_obj, part_flags,       \
                            num_cus, grid_out);
    B32(4, 4)
    B32(4, 8)
    B32(4, 16)
    B32(8, 16)
    B32(16, 16)
#undef B32
  }
  return hipErrorInvalidValue;
}

}  // namespace bumbar
