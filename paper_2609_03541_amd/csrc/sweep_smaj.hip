// Unbinned sweep over a sample-major copy of u, for 256 < K <= 1024 states.
//
// The copy holds u transposed: sample n is one contiguous row of Kp = 64 J
// values, J the smallest of 5, 6, 8, 10, 12, 14, 16 with K <= 64 J (states
// past K padded with +inf). One wavefront owns
// S = 2 samples at a time: lane l holds J states, V consecutive ones per
// 16-byte load (V = 2 in FP64, 4 in FP32 where J allows), so the
// per-sample log-sum-exp of Eq. (1), ln D_n = LSE_k(c_k - u_kn), is a
// register loop plus a 64-lane shuffle reduction, with no LDS traffic for the
// matrix and no barrier in the sample loop; the two samples' reduction chains
// interleave. With the exact sample maximum m_n:
//   e_kn = exp(c_k - u_kn - m_n),  D'_n = sum_{k sampled} e_kn,
//   acc_k += e_kn h_n / D'_n,      ln D_n = m_n + ln D'_n,
// so every element costs one exponential and u is read once, each wave load
// being 64 consecutive values of one sample (512 B in FP64). Waves are
// persistent and take sample pairs in grid order, so neighbouring waves read
// neighbouring rows. At the end each workgroup adds its waves' per-state
// sums through LDS (in wave order) and writes them state-major, the layout of
// the other sweeps' partials, for the same finaliser.
//
// Two arithmetic forms share the layout:
//  - FP64 (the FP64 copy, or an FP32 copy widened on load): the exponential is
//    the 64-entry table form (exp_nonpos_tab); the constants c_k and the
//    table sit in LDS.
//  - FP32 (mixed precision, FP32 or FP64 copy): the difference c_k - u_kn and the
//    sample maximum are taken in FP64, the shifted exponent is rounded to
//    FP32 and exponentiated with the hardware exp2; the column sums and the
//    per-lane state accumulators are FP32, the workgroup partials FP64.
#include <cmath>
#include <type_traits>

#include "bumbar_impl.h"
#include "devmath.h"

namespace bumbar {

constexpr int kSmajWaves = 4;
constexpr int kSmajS = 2;  // samples per wave iteration

// Slots per lane instantiated (J); a copy's rows are 64 J long for the
// smallest J that holds K states.
static const int kSmajJ[] = {5, 6, 8, 10, 12, 14, 16};
static int smaj_slots(int K) {
  for (int j : kSmajJ)
    if (K <= 64 * j) return j;
  return 0;
}
int smaj_row(int K) { return 64 * smaj_slots(K); }
size_t smaj_elems(int K, int64_t N) { return (size_t)smaj_row(K) * (size_t)N; }
bool sweep_smaj_supported(int K) { return K > 256 && K <= 1024; }

// Elements of one row a lane loads at once (16 bytes where J allows): slot j
// of lane l holds state V l + 64 V (j / V) + j % V.
template <int J, typename TI>
constexpr int smaj_vec() {
  return sizeof(TI) == 8 ? (J % 2 == 0 ? 2 : 1) : (J % 4 == 0 ? 4 : (J % 2 == 0 ? 2 : 1));
}
template <int J, typename TI>
__device__ __forceinline__ int smaj_state(int lane, int j) {
  constexpr int V = smaj_vec<J, TI>();
  return V * lane + 64 * V * (j / V) + j % V;
}

// Sample loop of one wave (see the file comment); MASKED: some state has
// N_k = 0 and is left out of D' (gm holds this lane's sampled slots).
template <int J, typename TI, bool F32A, bool MASKED, bool CHK>
__device__ __forceinline__ void smaj_loop(const TI* __restrict__ ut, int64_t N, int64_t n0,
                                          int64_t W, int lane, const double* __restrict__ c_sh,
                                          const float* __restrict__ c32_sh,
                                          const double* __restrict__ etab, unsigned gm,
                                          const double* __restrict__ h,
                                          double* __restrict__ logD,
                                          std::conditional_t<F32A, float, double> (&acc)[J],
                                          double& obj, unsigned& bad) {
  constexpr int S = kSmajS;
  constexpr int Kp = 64 * J;
  using TA = std::conditional_t<F32A, float, double>;
  for (int64_t nb = n0; nb < N; nb += W) {
    // rows past N re-read row N - 1 (their weight is zeroed below)
    constexpr int V = smaj_vec<J, TI>();
    typedef TI vT __attribute__((ext_vector_type(V)));
    TI x[S][J];
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const int64_t n = nb + i < N ? nb + i : N - 1;
      const TI* row = ut + n * Kp + V * lane;
#pragma unroll
      for (int jb = 0; jb < J / V; ++jb) {
        if constexpr (V == 1) {
          x[i][jb] = __builtin_nontemporal_load(row + 64 * jb);
        } else {
          const vT v = __builtin_nontemporal_load(reinterpret_cast<const vT*>(row + 64 * V * jb));
#pragma unroll
          for (int q = 0; q < V; ++q) x[i][jb * V + q] = v[q];
        }
      }
    }
    double m[S];
    if constexpr (F32A) {
      // the shift only has to be near the maximum: taken in FP32 (nothing
      // is held for the second pass, which recomputes the FP64 difference)
      float m32[S];
#pragma unroll
      for (int i = 0; i < S; ++i) m32[i] = -INFINITY;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const float cj = c32_sh[smaj_state<J, TI>(lane, j)];
#pragma unroll
        for (int i = 0; i < S; ++i) m32[i] = fmaxf(m32[i], cj - (float)x[i][j]);
      }
#pragma unroll
      for (int off = 1; off < 64; off <<= 1)
#pragma unroll
        for (int i = 0; i < S; ++i) m32[i] = fmaxf(m32[i], __shfl_xor(m32[i], off, 64));
#pragma unroll
      for (int i = 0; i < S; ++i) m[i] = m32[i] == -INFINITY ? 0.0 : (double)m32[i];
    } else {
      double chk = 0.0;
#pragma unroll
      for (int i = 0; i < S; ++i) m[i] = -INFINITY;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const double cj = c_sh[smaj_state<J, TI>(lane, j)];
#pragma unroll
        for (int i = 0; i < S; ++i) {
          const double a = cj - (double)x[i][j];
          m[i] = fmax(m[i], a);
          if constexpr (CHK) chk += a;  // NaN if any u is NaN (padding gives -inf, not NaN)
        }
      }
      if (CHK && chk != chk) bad |= FLAG_NAN;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1)
#pragma unroll
        for (int i = 0; i < S; ++i) m[i] = fmax(m[i], __shfl_xor(m[i], off, 64));
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (m[i] == -INFINITY) m[i] = 0.0;
    }
    TA e[S][J], d[S];
#pragma unroll
    for (int i = 0; i < S; ++i) d[i] = 0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const double cj = c_sh[smaj_state<J, TI>(lane, j)];
#pragma unroll
      for (int i = 0; i < S; ++i) {
        const double t = cj - (double)x[i][j] - m[i];
        if constexpr (F32A)
          e[i][j] = __builtin_amdgcn_exp2f((float)t * 1.44269504088896341f);
        else
          e[i][j] = exp_nonpos_tab(t, etab);
        if constexpr (MASKED)
          d[i] += ((gm >> j) & 1u) ? e[i][j] : (TA)0;
        else
          d[i] += e[i][j];  // padding states contribute exp(-inf) = 0
      }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1)
#pragma unroll
      for (int i = 0; i < S; ++i) d[i] += __shfl_xor(d[i], off, 64);
    TA w[S];
    double hl = 1.0, ml = m[0], dl = (double)d[0];
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const int64_t n = nb + i;
      const bool valid = n < N;
      const double hn = (h && valid) ? h[n] : 1.0;
      const double dd = (double)d[i];
      if constexpr (F32A) {
        if (valid && !(d[i] >= 1e-30f && d[i] <= 1e30f)) bad |= FLAG_COL;
        w[i] = valid ? (float)hn / d[i] : 0.0f;
      } else {
        if (valid && !(dd >= 1e-300 && dd <= 1e300)) bad |= FLAG_COL;
        w[i] = valid ? hn * rcp_nr(dd) : 0.0;
      }
      if (lane == i) {
        hl = hn;
        ml = m[i];
        dl = dd;
      }
    }
    // ln D_n of the S samples in one masked pass: lane i takes sample i
    if (lane < S && nb + lane < N) {
      const double l = ml + log_ge1(dl);
      if (logD) logD[nb + lane] = l;
      obj = __builtin_fma(hl, l, obj);
    }
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int i = 0; i < S; ++i) {
        if constexpr (F32A)
          acc[j] = __builtin_fmaf(e[i][j], w[i], acc[j]);
        else
          acc[j] = __builtin_fma(e[i][j], w[i], acc[j]);
      }
  }
}

// CHK: look for NaN in every element (a copy made by the caller); a copy made
// by the solve was checked once by the copy kernel.
template <int J, typename TI, bool F32A, bool CHK>
__global__ void __launch_bounds__(kSmajWaves * 64)
    sweep_smaj_kernel(const TI* __restrict__ ut, int K, int64_t N, const double* __restrict__ cst,
                      const double* __restrict__ gk, const double* __restrict__ h,
                      double* __restrict__ logD, double* __restrict__ part,
                      double* __restrict__ part_obj, unsigned* __restrict__ part_flags) {
  constexpr int Kp = 64 * J;
  using TA = std::conditional_t<F32A, float, double>;
  __shared__ double red[kSmajWaves / 2][Kp];
  __shared__ double c_sh[Kp];
  __shared__ float c32_sh[F32A ? Kp : 1];
  __shared__ double etab[64];
  __shared__ double ored[kSmajWaves];
  __shared__ unsigned fl;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) fl = 0u;
  for (int k = threadIdx.x; k < Kp; k += kSmajWaves * 64) {
    const double c = k < K ? cst[k] : -INFINITY;
    c_sh[k] = c;
    if constexpr (F32A) c32_sh[k] = (float)c;
  }
  if (threadIdx.x < 64) etab[threadIdx.x] = kExp2Frac64[threadIdx.x];
  TA acc[J];
  unsigned gm = 0u, valid_bits = 0u;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int k = smaj_state<J, TI>(lane, j);
    if (k < K) valid_bits |= 1u << j;
    if (k < K && gk[k] != 0.0) gm |= 1u << j;
    acc[j] = 0;
  }
  // any state with N_k = 0 in the problem? (uniform over the block; the
  // barrier also publishes c_sh and etab)
  const bool masked = __syncthreads_or(gm != valid_bits) != 0;
  double obj = 0.0;
  unsigned bad = 0u;
  const int64_t W = (int64_t)gridDim.x * kSmajWaves * kSmajS;
  const int64_t n0 = ((int64_t)blockIdx.x * kSmajWaves + wave) * kSmajS;
  if (masked)
    smaj_loop<J, TI, F32A, true, CHK>(ut, N, n0, W, lane, c_sh, c32_sh, etab, gm, h, logD, acc,
                                      obj, bad);
  else
    smaj_loop<J, TI, F32A, false, CHK>(ut, N, n0, W, lane, c_sh, c32_sh, etab, gm, h, logD, acc,
                                       obj, bad);
  // per-state sums of the workgroup, waves in order through LDS in two
  // halves (half the LDS, so more workgroups fit a CU):
  // v_k = ((a0 + a1) + a2) + a3
  constexpr int kHalf = kSmajWaves / 2;
  constexpr int kPer = (Kp + kSmajWaves * 64 - 1) / (kSmajWaves * 64);
  if (wave < kHalf) {
#pragma unroll
    for (int j = 0; j < J; ++j) red[wave][smaj_state<J, TI>(lane, j)] = (double)acc[j];
  }
  // objective: lanes 0 .. S-1 of each wave hold its parts
  double o = obj;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) o += __shfl_xor(o, off, 64);
  if (lane == 0) ored[wave] = o;
  if (bad) atomicOr(&fl, bad);
  __syncthreads();
  double t[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int k = threadIdx.x + q * kSmajWaves * 64;
    t[q] = 0.0;
    if (k < K) {
      t[q] = red[0][k];
#pragma unroll
      for (int wv = 1; wv < kHalf; ++wv) t[q] += red[wv][k];
    }
  }
  __syncthreads();
  if (wave >= kHalf) {
#pragma unroll
    for (int j = 0; j < J; ++j) red[wave - kHalf][smaj_state<J, TI>(lane, j)] = (double)acc[j];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int k = threadIdx.x + q * kSmajWaves * 64;
    if (k < K) {
      double v = t[q];
#pragma unroll
      for (int wv = 0; wv < kHalf; ++wv) v += red[wv][k];
      part[(int64_t)k * gridDim.x + blockIdx.x] = v;
    }
  }
  if (threadIdx.x == 0) {
    double ob = ored[0];
#pragma unroll
    for (int wv = 1; wv < kSmajWaves; ++wv) ob += ored[wv];
    part_obj[blockIdx.x] = ob;
    part_flags[blockIdx.x] = fl;
  }
}

template <int J, typename TI, bool F32A, bool CHK>
static hipError_t launch_smaj_t(hipStream_t s, const TI* ut, int K, int64_t N, const double* cst,
                                const double* gk, const double* h, double* logD, double* part,
                                double* part_obj, unsigned* part_flags, int num_cus,
                                int* grid_out) {
  auto kern = sweep_smaj_kernel<J, TI, F32A, CHK>;
  // resident workgroups per CU of this instantiation (queried once, thread-safe)
  static const int per_cu = [&] {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, kSmajWaves * 64, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    return nb;
  }();
  int64_t g = (int64_t)num_cus * per_cu;
  const int64_t need = (N + kSmajWaves * kSmajS - 1) / (kSmajWaves * kSmajS);
  if (g > need) g = need;
  if (g > sweep_max_grid(num_cus)) g = sweep_max_grid(num_cus);
  if (g < 1) g = 1;
  *grid_out = (int)g;
  hipLaunchKernelGGL(kern, dim3((unsigned)g), dim3(kSmajWaves * 64), 0, s, ut, K, N, cst, gk, h,
                     logD, part, part_obj, part_flags);
  return hipGetLastError();
}

hipError_t launch_sweep_smaj(hipStream_t s, const void* ut, bool f32, bool f32_arith,
                             bool nan_check, int K, int64_t N, const double* cst,
                             const double* gk, const double* h, double* logD, double* part,
                             double* part_obj, unsigned* part_flags, int num_cus, int* grid_out) {
  if (!sweep_smaj_supported(K)) return hipErrorInvalidValue;
  // the FP32 stage runs only over the solve's own (checked) copy
  if (f32_arith && nan_check) return hipErrorInvalidValue;
  const int J = smaj_slots(K);
  const float* uf = reinterpret_cast<const float*>(ut);
  const double* ud = reinterpret_cast<const double*>(ut);
#define BUMBAR_SMAJ_ARGS K, N, cst, gk, h, logD, part, part_obj, part_flags, num_cus, grid_out
#define BUMBAR_SMAJ(jj)                                                                        \
  if (J == jj) {                                                                               \
    if (f32_arith)                                                                             \
      return f32 ? launch_smaj_t<jj, float, true, false>(s, uf, BUMBAR_SMAJ_ARGS)              \
                 : launch_smaj_t<jj, double, true, false>(s, ud, BUMBAR_SMAJ_ARGS);            \
    if (nan_check)                                                                             \
      return f32 ? launch_smaj_t<jj, float, false, true>(s, uf, BUMBAR_SMAJ_ARGS)              \
                 : launch_smaj_t<jj, double, false, true>(s, ud, BUMBAR_SMAJ_ARGS);            \
    return f32 ? launch_smaj_t<jj, float, false, false>(s, uf, BUMBAR_SMAJ_ARGS)               \
               : launch_smaj_t<jj, double, false, false>(s, ud, BUMBAR_SMAJ_ARGS);             \
  }
  BUMBAR_SMAJ(5)
  BUMBAR_SMAJ(6)
  BUMBAR_SMAJ(8)
  BUMBAR_SMAJ(10)
  BUMBAR_SMAJ(12)
  BUMBAR_SMAJ(14)
  BUMBAR_SMAJ(16)
#undef BUMBAR_SMAJ
#undef BUMBAR_SMAJ_ARGS
  return hipErrorInvalidValue;
}

// Transpose u (K x N, row stride ld) into the sample-major copy (N x Kp,
// states past K = +inf) through 64 x 64 LDS tiles: both the reads (along n)
// and the writes (along k) are coalesced.
// With nan_flag, a NaN anywhere in u sets *nan_flag (the solve checks its
// copy once here instead of in every sweep).
template <typename TI>
__global__ void __launch_bounds__(256)
    smaj_copy_kernel(const TI* __restrict__ u, int64_t ld, int K, int64_t N, int Kp,
                     TI* __restrict__ ut, unsigned* __restrict__ nan_flag) {
  __shared__ TI tile[64][65];
  const int64_t n0 = (int64_t)blockIdx.x * 64;
  const int k0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  bool nan_seen = false;
  for (int r = ty; r < 64; r += 4) {
    const int k = k0 + r;
    const int64_t n = n0 + tx;
    const TI v = (k < K && n < N) ? u[(int64_t)k * ld + n] : (TI)INFINITY;
    nan_seen = nan_seen || v != v;
    tile[r][tx] = v;
  }
  if (__syncthreads_or(nan_seen) && nan_flag && threadIdx.x == 0) atomicOr(nan_flag, 1u);
  for (int r = ty; r < 64; r += 4) {
    const int64_t n = n0 + r;
    const int k = k0 + tx;
    if (n < N && k < Kp) ut[n * Kp + k] = tile[tx][r];
  }
}

hipError_t launch_smaj_copy(hipStream_t s, const void* u, bool f32, int64_t ld, int K, int64_t N,
                            void* ut, unsigned* nan_flag) {
  const int Kp = smaj_row(K);
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)(Kp / 64));
  if (f32)
    hipLaunchKernelGGL(smaj_copy_kernel<float>, grid, dim3(256), 0, s,
                       reinterpret_cast<const float*>(u), ld, K, N, Kp,
                       reinterpret_cast<float*>(ut), nan_flag);
  else
    hipLaunchKernelGGL(smaj_copy_kernel<double>, grid, dim3(256), 0, s,
                       reinterpret_cast<const double*>(u), ld, K, N, Kp,
                       reinterpret_cast<double*>(ut), nan_flag);
  return hipGetLastError();
}

}  // namespace bumbar
