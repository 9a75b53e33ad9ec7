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
#include <hip/hip_cooperative_groups.h>


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

// ---- batches of binned steps in one cooperative launch --------------------
//
// A batch of T self-consistent steps (Eq. (1) with the bin counts h_n,
// Algorithm 1) on a level materialised in the sample-major layout (FP64),
// 256 < K <= 1024. As separate launches each step is a sweep, a reduction of
// the per-state partials and a single-workgroup finaliser: three dependent
// launches whose fixed costs, not the level's few hundred kilobytes, set the
// step time. Here the grid is co-resident (cooperative launch) and a step is
//   sweep (as sweep_smaj_kernel: workgroup partials of every state)
//   -- grid barrier --
//   per-state sums S_k over the workgroup partials (T lanes per state, a
//   fixed xor butterfly), f_un_k = ln N'_k + f_k - ln S_k; every workgroup
//   also sums state 0 itself (the same lanes' order, so the same bits) for
//   the gauge f_new = f_un - f_un_0; iterate and per-workgroup scalars out
//   -- grid barrier --
// and after the last step the per-workgroup scalars of every step are added
// in workgroup order (Eq. (2) relative step, max |delta f|, objective,
// gradient norm, flags), a wave per value, the steps spread over the
// workgroups: off the steps' critical path, since the host reads the
// scalars only after the batch.
// Outputs per step are those of a sweep and its finaliser (f_hist row i,
// scal[i], ln D of the level); after the batch cst, gk and lnNp as the
// constants of a sweep at the last iterate, ln S and S of the last step.
// Measured on one MI355X it does not beat the per-step kernels (c2 ladder:
// 97 against 54 us per binned step; K = 1000, N = 4e4: 27 against 24): a
// grid barrier across the eight XCDs costs about as much as a kernel
// boundary, so the solve uses it only when asked (grid_batches = 1).
namespace {
constexpr int kBatchVals = 8;  // per-workgroup scalars: obj, flags, gsq, minS, mdf, rs, nf, pad

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ unsigned wave_or(unsigned v) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) v |= __shfl_xor(v, off, 64);
  return v;
}

// S_k summed by the T consecutive lanes starting at a multiple of T: lane c
// adds partials c, c + T, ... in order, then a fixed butterfly over the T
// lanes (every lane of the group gets the sum).
__device__ __forceinline__ double state_sum(const double* __restrict__ pk, int G, int T, int c) {
  // eight loads in flight per round trip
  double a[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) a[q] = 0.0;
  int p = c;
  for (; p + 7 * T < G; p += 8 * T) {
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] += pk[p + q * T];
  }
  for (; p < G; p += T) a[0] += pk[p];
  double v = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  for (int off = 1; off < T; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace

template <int J>
__global__ void __launch_bounds__(kSmajWaves * 64)
    smaj_batch_kernel(const double* __restrict__ ut, int K, int64_t P,
                      const double* __restrict__ h, const int64_t* __restrict__ Nk,
                      const double* __restrict__ f_in, int T, int TL,
                      double* __restrict__ f_hist, SweepScalars* __restrict__ scal,
                      double* __restrict__ logD, double* __restrict__ lnS_out,
                      double* __restrict__ S_out, double* __restrict__ cst,
                      double* __restrict__ gk_out, double* __restrict__ lnNp_out,
                      double* __restrict__ part, double* __restrict__ wsc) {
  using TI = double;
  constexpr int Kp = 64 * J;
  constexpr int NT = kSmajWaves * 64;
  __shared__ double red[kSmajWaves / 2][Kp];
  __shared__ double c_sh[Kp];
  __shared__ double lnNp_sh[Kp];
  __shared__ double etab[64];
  __shared__ double wred[kSmajWaves][7];
  __shared__ double g0_sh;
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  const int G = gridDim.x, b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int k = tid; k < Kp; k += NT) {
    const int64_t n = k < K ? Nk[k] : 0;
    lnNp_sh[k] = n > 0 ? log((double)n) : 0.0;
  }
  if (tid < 64) etab[tid] = kExp2Frac64[tid];
  unsigned gm = 0u, valid_bits = 0u;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int k = smaj_state<J, TI>(lane, j);
    if (k < K) valid_bits |= 1u << j;
    if (k < K && Nk[k] > 0) gm |= 1u << j;
  }
  const bool masked = __syncthreads_or(gm != valid_bits) != 0;
  const int64_t W = (int64_t)G * kSmajWaves * kSmajS;
  const int64_t n0 = ((int64_t)b * kSmajWaves + wave) * kSmajS;
  constexpr int kHalf = kSmajWaves / 2;
  constexpr int kPer = (Kp + NT - 1) / NT;
  for (int it = 0; it < T; ++it) {
    const double* fp = it == 0 ? f_in : f_hist + (int64_t)(it - 1) * K;
    double* ws = wsc + (int64_t)it * G * kBatchVals;
    // ---- sweep at fp ----
    for (int k = tid; k < Kp; k += NT) c_sh[k] = k < K ? lnNp_sh[k] + fp[k] : -INFINITY;
    __syncthreads();
    double acc[J];
#pragma unroll
    for (int j = 0; j < J; ++j) acc[j] = 0.0;
    double obj = 0.0;
    unsigned bad = 0u;
    if (masked)
      smaj_loop<J, TI, false, true, false>(ut, P, n0, W, lane, c_sh, nullptr, etab, gm, h, logD,
                                           acc, obj, bad);
    else
      smaj_loop<J, TI, false, false, false>(ut, P, n0, W, lane, c_sh, nullptr, etab, gm, h, logD,
                                            acc, obj, bad);
    if (wave < kHalf) {
#pragma unroll
      for (int j = 0; j < J; ++j) red[wave][smaj_state<J, TI>(lane, j)] = acc[j];
    }
    const double o = wave_sum(obj);
    const unsigned fw = wave_or(bad);
    if (lane == 0) {
      wred[wave][0] = o;
      wred[wave][1] = (double)fw;
    }
    __syncthreads();
    double t[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int k = tid + q * NT;
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
      for (int j = 0; j < J; ++j) red[wave - kHalf][smaj_state<J, TI>(lane, j)] = acc[j];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int k = tid + q * NT;
      if (k < K) {
        double v = t[q];
#pragma unroll
        for (int wv = 0; wv < kHalf; ++wv) v += red[wv][k];
        part[(int64_t)k * G + b] = v;
      }
    }
    if (tid == 0) {
      double ob = wred[0][0];
      unsigned fl = (unsigned)wred[0][1];
      for (int wv = 1; wv < kSmajWaves; ++wv) {
        ob += wred[wv][0];
        fl |= (unsigned)wred[wv][1];
      }
      ws[(int64_t)b * kBatchVals + 0] = ob;
      ws[(int64_t)b * kBatchVals + 1] = (double)fl;
    }
    grid.sync();
    // ---- per-state sums, new f, gauge ----
    if (wave == 0) {
      const double S0 = lane < TL ? state_sum(part, G, TL, lane) : 0.0;
      if (lane == 0) g0_sh = lnNp_sh[0] + fp[0] - log(S0);
    }
    __syncthreads();
    const double fu0 = g0_sh;
    double gsq = 0.0, minS = INFINITY, mdf = 0.0, rs = 0.0, nf = 0.0;
    unsigned fl = 0u;
    const int64_t gl = (int64_t)b * NT + tid;
    const int64_t stride = (int64_t)G * NT / TL;
    for (int64_t k = gl / TL; k < K; k += stride) {
      const double S = state_sum(part + k * G, G, TL, (int)(gl % TL));
      if (gl % TL != 0) continue;
      const double lnS = log(S);
      const double fo = fp[k];
      const double fun = lnNp_sh[k] + fo - lnS;
      if (!(S >= 1e-290 && S <= 1e290)) fl |= FLAG_STATE;
      if (fun != fun) fl |= FLAG_NAN;
      const double fn = fun - fu0;
      f_hist[(int64_t)it * K + k] = fn;
      const int64_t nk = Nk[k];
      if (nk > 0) {
        const double g = S - (double)nk;
        gsq += g * g;
        minS = fmin(minS, S);
      }
      double df = fabs(fn - fo);
      if (df != df) df = INFINITY;
      mdf = fmax(mdf, df);
      if (k >= 1) {
        double r;
        if (fo != 0.0)
          r = fabs(fn / fo - 1.0);
        else
          r = (fn == 0.0) ? 0.0 : INFINITY;
        if (r != r) r = INFINITY;
        rs = fmax(rs, r);
      }
      nf = __builtin_fma(-(double)nk, fo, nf);
      if (it == T - 1) {
        lnS_out[k] = lnS;
        S_out[k] = S;
        cst[k] = lnNp_sh[k] + fn;
        gk_out[k] = nk > 0 ? 1.0 : 0.0;
        lnNp_out[k] = lnNp_sh[k];
      }
    }
    // workgroup scalars: waves in order
    gsq = wave_sum(gsq);
    minS = wave_min(minS);
    mdf = wave_max(mdf);
    rs = wave_max(rs);
    nf = wave_sum(nf);
    fl = wave_or(fl);
    if (lane == 0) {
      wred[wave][0] = gsq;
      wred[wave][1] = minS;
      wred[wave][2] = mdf;
      wred[wave][3] = rs;
      wred[wave][4] = nf;
      wred[wave][5] = (double)fl;
    }
    __syncthreads();
    if (tid == 0) {
      double v[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) v[q] = wred[0][q];
      unsigned f2 = (unsigned)v[5];
      for (int wv = 1; wv < kSmajWaves; ++wv) {
        v[0] += wred[wv][0];
        v[1] = fmin(v[1], wred[wv][1]);
        v[2] = fmax(v[2], wred[wv][2]);
        v[3] = fmax(v[3], wred[wv][3]);
        v[4] += wred[wv][4];
        f2 |= (unsigned)wred[wv][5];
      }
      double* slot = ws + (int64_t)b * kBatchVals;
      slot[2] = v[0];
      slot[3] = v[1];
      slot[4] = v[2];
      slot[5] = v[3];
      slot[6] = v[4];
      slot[7] = (double)f2;
    }
    grid.sync();
  }
  // ---- the scalars of every step: step s on workgroup s mod G, value q on
  // wave q mod 4, lane l adding workgroups l, l + 64, ... then a butterfly ----
  __shared__ double sv[kBatchVals];
  for (int st = b; st < T; st += G) {
    const double* ws = wsc + (int64_t)st * G * kBatchVals;
    for (int q = wave; q < kBatchVals - 1; q += kSmajWaves) {
      // q: 0 obj (sum), 1 sweep flags (or), 2 gsq (sum), 3 minS (min),
      // 4 mdf (max), 5 rs (max), 6 nf (sum); the state flags (slot 7) go
      // with q = 1
      double v = (q == 3) ? INFINITY : 0.0;
      unsigned fo = 0u;
      for (int w = lane; w < G; w += 64) {
        const double x = ws[(int64_t)w * kBatchVals + q];
        if (q == 1)
          fo |= (unsigned)x | (unsigned)ws[(int64_t)w * kBatchVals + 7];
        else if (q == 3)
          v = fmin(v, x);
        else if (q == 4 || q == 5)
          v = fmax(v, x);
        else
          v += x;
      }
      if (q == 1)
        v = (double)wave_or(fo);
      else if (q == 3)
        v = wave_min(v);
      else if (q == 4 || q == 5)
        v = wave_max(v);
      else
        v = wave_sum(v);
      if (lane == 0) sv[q] = v;
    }
    __syncthreads();
    if (tid == 0) {
      SweepScalars sc;
      sc.max_df = sv[4];
      sc.rel_step = sv[5];
      sc.objective = sv[0] + sv[6];
      sc.grad_norm = sqrt(sv[2]);
      sc.min_S = sv[3];
      sc.flags = (unsigned)sv[1];
      sc.pad = 0u;
      scal[st] = sc;
    }
    __syncthreads();
  }
}

bool smaj_batch_supported(int K) { return sweep_smaj_supported(K); }

int64_t smaj_batch_scratch(int num_cus, int max_steps) {
  return (int64_t)max_steps * sweep_max_grid(num_cus) * kBatchVals;
}

template <int J>
static hipError_t launch_batch_t(hipStream_t s, const double* ut, int K, int64_t P,
                                 const double* h, const int64_t* Nk, const double* f_in, int T,
                                 double* f_hist, SweepScalars* scal, double* logD, double* lnS,
                                 double* S, double* cst, double* gk, double* lnNp, double* part,
                                 int part_cap, double* wsc, int num_cus) {
  auto kern = smaj_batch_kernel<J>;
  static const int per_cu = [&] {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, kSmajWaves * 64, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 0;
    return nb;
  }();
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  // co-resident grid (at most the occupancy limit), at least one wave's
  // sample pair per wave, within the partials' and the scalars' capacity
  int64_t g = (int64_t)num_cus * per_cu;
  const int64_t need = (P + kSmajWaves * kSmajS - 1) / (kSmajWaves * kSmajS);
  if (g > need) g = need;
  if (g > part_cap) g = part_cap;
  if (g > sweep_max_grid(num_cus)) g = sweep_max_grid(num_cus);
  if (g < 1) g = 1;
  int G = (int)g;
  // lanes per state in the per-state sums: a power of two up to 64, as many
  // as the grid's threads allow for K states
  int TL = 1;
  while (TL < 64 && (int64_t)2 * TL * K <= (int64_t)G * kSmajWaves * 64) TL *= 2;
  void* args[] = {&ut, &K, &P, &h, &Nk, &f_in, &T, &TL, &f_hist, &scal, &logD, &lnS, &S,
                  &cst, &gk, &lnNp, &part, &wsc};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3((unsigned)G),
                                    dim3(kSmajWaves * 64), args, 0, s);
}

hipError_t launch_smaj_batch(hipStream_t s, const double* ut, int K, int64_t P, const double* h,
                             const int64_t* Nk, const double* f_in, int T, double* f_hist,
                             SweepScalars* scal, double* logD, double* lnS, double* S,
                             double* cst, double* gk, double* lnNp, double* part, int part_cap,
                             double* wsc, int wsc_steps, int num_cus) {
  if (!smaj_batch_supported(K) || T < 1 || T > wsc_steps || P < 1 || !ut || !Nk || !f_in ||
      !f_hist || !scal ||
      !logD || !lnS || !S || !cst || !gk || !lnNp || !part || part_cap < 1 || !wsc)
    return hipErrorInvalidValue;
  const int J = smaj_slots(K);
#define BUMBAR_BATCH(jj)                                                                      \
  if (J == jj)                                                                                \
    return launch_batch_t<jj>(s, ut, K, P, h, Nk, f_in, T, f_hist, scal, logD, lnS, S, cst, gk, \
                              lnNp, part, part_cap, wsc, num_cus);
  BUMBAR_BATCH(5)
  BUMBAR_BATCH(6)
  BUMBAR_BATCH(8)
  BUMBAR_BATCH(10)
  BUMBAR_BATCH(12)
  BUMBAR_BATCH(14)
  BUMBAR_BATCH(16)
#undef BUMBAR_BATCH
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
