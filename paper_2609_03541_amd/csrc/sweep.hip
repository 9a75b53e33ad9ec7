// Sweep kernels of the MBAR self-consistent iteration on gfx950.
//
// One sweep evaluates, for the current free energies f (Section 2, Eq. (1) in
// its unbinned limit, or binned with per-column multiplicities h_p):
//   ln D_n  = ln sum_{k: N_k>0} N_k exp(f_k - u_kn)
//   S_i     = sum_n h_n N_i exp(f_i - u_in - ln D_n)          (h_n = 1 unbinned)
//   f_new_i = ln N'_i + f_i - ln S_i                            (then gauge f_0 = 0)
// which is f_new_i = -ln sum_n h_n exp(-u_in - ln D_n).
//
// Fast path (sweep_fast): a persistent workgroup owns a K x TN column tile per
// iteration, held in registers. With a_kn = c_k - u_kn (c_k = ln N'_k + f_k):
//   pass 1: m_n = max_k a_kn                   (exact column shift)
//   pass 2: e_kn = exp(a_kn - m_n), D'_n = sum_k g_k e_kn
//   pass 3: acc_k += e_kn * h_n / D'_n         (per-thread, per-state accumulator)
// so u_kn is read from HBM once and each element costs one exponential. The
// per-state accumulators are reduced across lanes and written once per
// workgroup; the finaliser adds the workgroup partials in a fixed order, so a
// sweep is deterministic (no floating-point atomics anywhere).
//
// The shift m_n makes every e_kn <= 1 (no overflow). A state whose every
// weight is below the double range (a far-off starting f) would make S_i
// underflow; the finaliser flags that and the host reruns the sweep on the
// robust two-pass path, which keeps an exact per-state log-sum-exp.
#include <cfloat>
#include <cmath>
#include <type_traits>
#include <cstdio>
#include <cstdlib>

#include "bumbar_impl.h"
#include "devmath.h"

namespace bumbar {

__device__ __forceinline__ double shfl_xor_d(double v, int mask) { return __shfl_xor(v, mask, 64); }

// ---------------------------------------------------------------------------
// Fast single-pass sweep.
//   NW   waves per workgroup         LPR  lanes along a row segment
//   CPL  columns per lane            ROWS rows (states) per thread
// Thread t: column lane lc = t % LPR, row group rg = t / LPR; it owns rows
// k = rg + RG * j (j < ROWS) and columns col0 .. col0 + CPL - 1 of each tile.
// Rows past K read row K - 1 (always in bounds) and are masked by c_k = -inf,
// so the main loop has no per-row branches; the last, partial column tile
// takes a separate guarded path.
// ---------------------------------------------------------------------------
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
constexpr double kLog2e = 1.4426950408889634;

template <int NW, int LPR, int CPL, int ROWS>
struct SweepTile {
  static constexpr int NT = NW * 64;
  static constexpr int RG = NT / LPR;
  static constexpr int TN = LPR * CPL;
};

// Load this thread's ROWS x CPL elements of column tile t. Padding rows
// (j >= rows_here) re-read the thread's last valid row (c_k = -inf masks
// them); in the TAIL tile columns past N re-read column N - 1 (their weight is
// zeroed). The row offsets are opaque to the compiler so every load is
// unconditional: no branch and no reuse of another row's value, hence no wait
// on an earlier load before the next is issued.
template <int NW, int LPR, int CPL, int ROWS, bool VEC, bool TAIL, typename TI>
__device__ __forceinline__ void tile_load(double (&a)[ROWS][CPL], const TI* __restrict__ rowp,
                                          int64_t rstride, int rows_here, int64_t t, int64_t N,
                                          int lc) {
  constexpr int TN = SweepTile<NW, LPR, CPL, ROWS>::TN;
  const int64_t col0 = t * TN + (int64_t)lc * CPL;
#pragma unroll
  for (int j = 0; j < ROWS; ++j) {
    int64_t roff = (int64_t)(j < rows_here ? j : (rows_here > 0 ? rows_here - 1 : 0)) * rstride;
    asm volatile("" : "+v"(roff));
    const TI* p = rowp + roff + t * TN;
    if constexpr (!TAIL && VEC && CPL == 2) {
      // u is streamed once per sweep: non-temporal loads (c1 sweep 181 -> 171 us);
      // FP32 storage is widened exactly on load
      if constexpr (std::is_same<TI, double>::value) {
        const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
        a[j][0] = v.x;
        a[j][1] = v.y;
      } else {
        const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
        a[j][0] = (double)v.x;
        a[j][1] = (double)v.y;
      }
    } else if constexpr (!TAIL) {
#pragma unroll
      for (int i = 0; i < CPL; ++i) a[j][i] = (double)p[i];
    } else {
#pragma unroll
      for (int i = 0; i < CPL; ++i) {
        const int64_t off = (col0 + i < N) ? (int64_t)i : (N - 1 - col0);
        a[j][i] = (double)p[off];
      }
    }
  }
}

// The three passes over a loaded tile (see the file comment). red1 / red2
// are read by every wave in the ln D step at the end, so a caller that runs
// tiles back to back without a barrier between them alternates two copies of
// them (a wave may start the next tile's pass 1 while another is still
// reading this tile's).
template <int NW, int LPR, int CPL, int ROWS, bool TAIL, bool MASKED, int SG, bool F32A = false>
__device__ __forceinline__ void tile_compute(double (&a)[ROWS][CPL], int64_t t, int64_t N, int lc,
                                             int rg, int wave, int rgw,
                                             const double* __restrict__ c_sh, unsigned smask,
                                             const double* __restrict__ h,
                                             double* __restrict__ logD,
                                             double (*red1)[LPR * CPL], double (*red2)[LPR * CPL],
                                             double* acc, double& obj, unsigned& bad) {
  using TL = SweepTile<NW, LPR, CPL, ROWS>;
  constexpr int RG = TL::RG;
  constexpr int TN = TL::TN;
  const int64_t col0 = t * TN + (int64_t)lc * CPL;
  // opaque copies: re-read c_k from LDS each tile rather than pin ROWS
  // registers to it
  int rgo = rg;
  unsigned sm = smask;
  asm volatile("" : "+v"(rgo), "+v"(sm));
  // ---- pass 1: a = c - u and the column maximum ----
  double cm[CPL], chk = 0.0;
#pragma unroll
  for (int i = 0; i < CPL; ++i) cm[i] = -INFINITY;
#pragma unroll
  for (int j = 0; j < ROWS; ++j) {
    const double c = c_sh[rgo + RG * j];
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      a[j][i] = c - a[j][i];
      cm[i] = fmax(cm[i], a[j][i]);
      chk += a[j][i];  // NaN if any u is NaN (or -inf): the max would drop it
    }
  }
  if (chk != chk) bad |= FLAG_NAN;
#pragma unroll
  for (int i = 0; i < CPL; ++i) {
#pragma unroll
    for (int off = LPR; off < 64; off <<= 1) cm[i] = fmax(cm[i], __shfl_xor(cm[i], off, 64));
    if (rgw == 0) red1[wave][lc * CPL + i] = cm[i];
  }
  __syncthreads();
  double m[CPL];
#pragma unroll
  for (int i = 0; i < CPL; ++i) {
    double v = red1[0][lc * CPL + i];
#pragma unroll
    for (int w = 1; w < NW; ++w) v = fmax(v, red1[w][lc * CPL + i]);
    m[i] = (v == -INFINITY) ? 0.0 : v;
  }
  // ---- pass 2: e = exp(a - m) and the column sum over sampled states ----
  double ds[CPL];
#pragma unroll
  for (int i = 0; i < CPL; ++i) ds[i] = 0.0;
#pragma unroll
  for (int j = 0; j < ROWS; ++j) {
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      if constexpr (F32A)  // FP32 stage of mixed precision: FP32 hardware exp2, FP64 sums
        a[j][i] = (double)__builtin_amdgcn_exp2f((float)((a[j][i] - m[i]) * kLog2e));
      else
        a[j][i] = exp_nonpos(a[j][i] - m[i]);
      if constexpr (MASKED) {
        ds[i] = ((sm >> j) & 1u) ? ds[i] + a[j][i] : ds[i];
      } else {
        ds[i] += a[j][i];
      }
    }
    // schedule the exponentials in groups of SG rows (0: no grouping); a
    // group boundary bounds register pressure at the cost of fewer
    // independent chains in flight
    if constexpr (SG > 0) {
      if ((j + 1) % SG == 0) __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int i = 0; i < CPL; ++i) {
#pragma unroll
    for (int off = LPR; off < 64; off <<= 1) ds[i] += __shfl_xor(ds[i], off, 64);
    if (rgw == 0) red2[wave][lc * CPL + i] = ds[i];
  }
  __syncthreads();
  double w[CPL];
#pragma unroll
  for (int i = 0; i < CPL; ++i) {
    double D = red2[0][lc * CPL + i];
#pragma unroll
    for (int wv = 1; wv < NW; ++wv) D += red2[wv][lc * CPL + i];
    const int64_t n = col0 + i;
    const bool valid = !TAIL || n < N;
    const double hn = (h != nullptr && valid) ? h[n] : 1.0;
    w[i] = valid ? hn * rcp_nr(D) : 0.0;
    if (valid && !(D >= 1e-300 && D <= 1e300)) bad |= FLAG_COL;
  }
  // ---- pass 3: per-state accumulation of e * h / D' ----
#pragma unroll
  for (int j = 0; j < ROWS; ++j)
#pragma unroll
    for (int i = 0; i < CPL; ++i) acc[j] = __builtin_fma(a[j][i], w[i], acc[j]);
  // the tile values are dead from here on: do the logarithms now
  __builtin_amdgcn_sched_barrier(0);
  // ln D_n and the objective: wave v handles columns [v * CW, (v + 1) * CW),
  // one lane each, so every wave evaluates one logarithm per tile.
  {
    constexpr int CW = TN / NW;
    const int lane = threadIdx.x & 63;
    if (lane < CW) {
      const int col = wave * CW + lane;
      double mv = red1[0][col], Dv = red2[0][col];
#pragma unroll
      for (int wv = 1; wv < NW; ++wv) {
        mv = fmax(mv, red1[wv][col]);
        Dv += red2[wv][col];
      }
      if (mv == -INFINITY) mv = 0.0;
      const int64_t n = t * TN + col;
      if (!TAIL || n < N) {
        const double l = mv + log_ge1(Dv);
        if (logD != nullptr) logD[n] = l;
        obj = __builtin_fma(h != nullptr ? h[n] : 1.0, l, obj);
      }
    }
  }
}

// Tile loop over the full tiles of this block; with PF the next tile's loads
// are issued into a second register buffer before the current tile is
// processed (software prefetch), so HBM traffic overlaps the arithmetic.
// Successive tiles use alternating copies (par) of the reduction buffers.
template <int NW, int LPR, int CPL, int ROWS, bool VEC, bool MASKED, bool PF, int SG, typename TI,
          bool F32A>
__device__ __forceinline__ void tile_loop(const TI* __restrict__ base, int64_t rstride,
                                          int rows_here, int64_t nfull, int64_t N, int lc, int rg,
                                          int wave, int rgw, const double* __restrict__ c_sh,
                                          unsigned smask, const double* __restrict__ h,
                                          double* __restrict__ logD,
                                          double (*red1)[NW][LPR * CPL],
                                          double (*red2)[NW][LPR * CPL], int& par, double* acc,
                                          double& obj, unsigned& bad) {
  const int64_t G = gridDim.x;
  int64_t t = blockIdx.x;
  if constexpr (!PF) {
    for (; t < nfull; t += G) {
      double a[ROWS][CPL];
      tile_load<NW, LPR, CPL, ROWS, VEC, false, TI>(a, base, rstride, rows_here, t, N, lc);
      tile_compute<NW, LPR, CPL, ROWS, false, MASKED, SG, F32A>(a, t, N, lc, rg, wave, rgw, c_sh, smask, h,
                                                      logD, red1[par], red2[par], acc, obj, bad);
      par ^= 1;
    }
  } else {
    double a[ROWS][CPL], b[ROWS][CPL];
    if (t < nfull) tile_load<NW, LPR, CPL, ROWS, VEC, false, TI>(a, base, rstride, rows_here, t, N, lc);
    while (t < nfull) {
      const int64_t t1 = t + G;
      if (t1 < nfull) tile_load<NW, LPR, CPL, ROWS, VEC, false, TI>(b, base, rstride, rows_here, t1, N, lc);
      tile_compute<NW, LPR, CPL, ROWS, false, MASKED, SG, F32A>(a, t, N, lc, rg, wave, rgw, c_sh, smask, h,
                                                      logD, red1[par], red2[par], acc, obj, bad);
      par ^= 1;
      if (t1 >= nfull) break;
      const int64_t t2 = t1 + G;
      if (t2 < nfull) tile_load<NW, LPR, CPL, ROWS, VEC, false, TI>(a, base, rstride, rows_here, t2, N, lc);
      tile_compute<NW, LPR, CPL, ROWS, false, MASKED, SG, F32A>(b, t1, N, lc, rg, wave, rgw, c_sh, smask, h,
                                                      logD, red1[par], red2[par], acc, obj, bad);
      par ^= 1;
      t = t2;
    }
  }
}

template <int NW, int LPR, int CPL, int ROWS, bool VEC, bool PF, int SG, typename TI, bool F32A>
__global__ void __launch_bounds__(NW * 64)
    sweep_fast_kernel(const TI* __restrict__ u, int64_t ld, int K, int64_t N,
                      int64_t ntiles, const double* __restrict__ cst,
                      const double* __restrict__ gk, const double* __restrict__ h,
                      double* __restrict__ logD, double* __restrict__ part,
                      double* __restrict__ part_obj, unsigned* __restrict__ part_flags) {
  using TL = SweepTile<NW, LPR, CPL, ROWS>;
  constexpr int NT = TL::NT;
  constexpr int RG = TL::RG;
  constexpr int TN = TL::TN;
  __shared__ double red1[2][NW][TN];
  __shared__ double red2[2][NW][TN];
  __shared__ double c_sh[ROWS * RG];
  __shared__ double tr[ROWS * RG * (LPR + 1)];  // per-state lane sums at the end
  static_assert(LPR % 4 == 0, "lane sums are taken four at a time");
  __shared__ unsigned fl;

  const int tid = threadIdx.x;
  const int lc = tid % LPR;
  const int rg = tid / LPR;
  const int wave = tid >> 6;
  const int rgw = (tid & 63) / LPR;

  // per-state constants: c_k in LDS (-inf for padding rows), sampled flags as a
  // bitmask (used only when some state has N_k = 0)
  for (int k = tid; k < ROWS * RG; k += NT) c_sh[k] = (k < K) ? cst[k] : -INFINITY;
  if (tid == 0) fl = 0u;
  unsigned smask = 0u;
  double acc[ROWS];
#pragma unroll
  for (int j = 0; j < ROWS; ++j) {
    const int k = rg + RG * j;
    if (k < K && gk[k] != 0.0) smask |= 1u << j;
    acc[j] = 0.0;
  }
  // Pointer to this thread's first row (row 0 for a thread with no valid
  // row); its rows are RG apart. rows_here counts its rows below K.
  const int rows_here = (rg < K) ? (K - 1 - rg) / RG + 1 : 0;
  const TI* base = u + (int64_t)((rg < K) ? rg : 0) * ld + (int64_t)lc * CPL;
  const int64_t rstride = (int64_t)RG * ld;
  // any state with N_k = 0 among this block's rows? (uniform over the block)
  const unsigned valid_bits = (rows_here >= 32) ? 0xffffffffu : ((1u << rows_here) - 1u);
  const bool masked = __syncthreads_or(smask != valid_bits) != 0;

  double obj = 0.0;
  unsigned bad = 0;
  int par = 0;
  const int64_t nfull = N / TN;
  if (!masked)
    tile_loop<NW, LPR, CPL, ROWS, VEC, false, PF, SG, TI, F32A>(base, rstride, rows_here, nfull, N, lc, rg, wave,
                                                  rgw, c_sh, smask, h, logD, red1, red2, par, acc,
                                                  obj, bad);
  else
    tile_loop<NW, LPR, CPL, ROWS, VEC, true, false, 1, TI, F32A>(base, rstride, rows_here, nfull, N, lc, rg,
                                                    wave, rgw, c_sh, smask, h, logD, red1, red2,
                                                    par, acc, obj, bad);
  if (nfull < ntiles && blockIdx.x == (unsigned)(nfull % gridDim.x)) {
    double a[ROWS][CPL];
    tile_load<NW, LPR, CPL, ROWS, VEC, true, TI>(a, base, rstride, rows_here, nfull, N, lc);
    tile_compute<NW, LPR, CPL, ROWS, true, true, 1, F32A>(a, nfull, N, lc, rg, wave, rgw, c_sh, smask, h,
                                                 logD, red1[par], red2[par], acc, obj, bad);
  }

  // Each state's accumulators over the LPR lanes of its row group: through
  // LDS (rows padded by one against bank conflicts), then one thread per
  // state adds its LPR values in lane order. A butterfly of shuffles per
  // state would chain ROWS x log2(LPR) dependent LDS round trips instead.
#pragma unroll
  for (int j = 0; j < ROWS; ++j) tr[(rg + RG * j) * (LPR + 1) + lc] = acc[j];
  __syncthreads();
  for (int k = tid; k < K && k < ROWS * RG; k += NT) {
    const double* row = &tr[k * (LPR + 1)];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int l = 0; l < LPR; l += 4) {
      s0 += row[l];
      s1 += row[l + 1];
      s2 += row[l + 2];
      s3 += row[l + 3];
    }
    part[(int64_t)k * gridDim.x + blockIdx.x] = (s0 + s1) + (s2 + s3);  // state-major
  }
  // objective partial: sum over the block (wave butterflies, then waves in order)
  double o = obj;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) o += __shfl_xor(o, off, 64);
  __syncthreads();  // red1 is free again
  if ((tid & 63) == 0) red1[0][0][wave] = o;
  __syncthreads();
  if (tid == 0) {
    double ob = red1[0][0][0];
    for (int wv = 1; wv < NW; ++wv) ob += red1[0][0][wv];
    part_obj[blockIdx.x] = ob;
  }
  // flags: OR over the block in shared memory, then one plain store
  if (bad) atomicOr(&fl, bad);
  __syncthreads();
  if (tid == 0) part_flags[blockIdx.x] = fl;
}

// Launch configuration table: (NW, LPR, CPL, ROWS, PF, SG) by number of states.
struct FastCfg {
  int kmax, nw, lpr, cpl, rows, pf, sg;
};
static const FastCfg kCfgs[] = {
    {8, 4, 64, 2, 2, 1, 1},    {16, 4, 64, 2, 4, 1, 1},   {32, 4, 64, 2, 8, 1, 1},
    {56, 4, 32, 2, 7, 1, 1},   {64, 4, 32, 2, 8, 1, 1},   {104, 4, 32, 2, 13, 0, 0},
    {128, 4, 32, 2, 16, 0, 1},
    {256, 8, 32, 2, 16, 0, 1},
};
static const FastCfg* pick_cfg(int K) {
  for (const auto& c : kCfgs)
    if (K <= c.kmax) return &c;
  return nullptr;
}

bool sweep_fast_supported(int K) { return pick_cfg(K) != nullptr; }

int sweep_max_grid(int num_cus) { return num_cus * 8; }

template <int NW, int LPR, int CPL, int ROWS, int PF, int SG, typename TI, bool F32A = false>
static hipError_t launch_cfg(hipStream_t s, bool vec, const TI* u, int64_t ld, int K,
                             int64_t N, const double* cst, const double* gk, const double* h,
                             double* logD, double* part, double* part_obj, unsigned* pf,
                             int num_cus, int* grid_out) {
  constexpr int TN = LPR * CPL;
  const int64_t ntiles = (N + TN - 1) / TN;
  auto kv = sweep_fast_kernel<NW, LPR, CPL, ROWS, true, PF != 0, SG, TI, F32A>;
  auto ks = sweep_fast_kernel<NW, LPR, CPL, ROWS, false, PF != 0, SG, TI, F32A>;
  // resident workgroups per CU of this instantiation (queried once, thread-safe)
  static const int per_cu = [&] {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kv, NW * 64, 0) != hipSuccess || nb < 1)
      nb = 1;
    return nb;
  }();
  int64_t g = (int64_t)num_cus * per_cu;
  if (g > ntiles) g = ntiles;
  if (g > sweep_max_grid(num_cus)) g = sweep_max_grid(num_cus);
  if (g < 1) g = 1;
  *grid_out = (int)g;
  if (vec)
    hipLaunchKernelGGL(kv, dim3((unsigned)g), dim3(NW * 64), 0, s, u, ld, K, N, ntiles, cst, gk, h,
                       logD, part, part_obj, pf);
  else
    hipLaunchKernelGGL(ks, dim3((unsigned)g), dim3(NW * 64), 0, s, u, ld, K, N, ntiles, cst, gk, h,
                       logD, part, part_obj, pf);
  return hipGetLastError();
}

hipError_t launch_sweep_fast(hipStream_t s, const void* u, bool f32, bool f32_arith, int64_t ld,
                             int K, int64_t N, const double* cst, const double* gk,
                             const double* h, double* logD, double* part, double* part_obj,
                             unsigned* part_flags, int num_cus, int* grid_out) {
  const FastCfg* c = pick_cfg(K);
  if (!c) return hipErrorInvalidValue;
  if (f32_arith && !f32) return hipErrorInvalidValue;  // FP32 exponentials only over FP32 storage
  // two columns per load: 16 bytes in FP64, 8 bytes in FP32
  const uintptr_t al = f32 ? 7 : 15;
  const bool vec = ((reinterpret_cast<uintptr_t>(u) & al) == 0) && ((ld & 1) == 0);
  const double* ud = static_cast<const double*>(u);
  const float* uf = static_cast<const float*>(u);
#define BUMBAR_CFG(a, b, cc, d, e, f)                                                            \
  if (c->nw == a && c->lpr == b && c->cpl == cc && c->rows == d && c->pf == e && c->sg == f) {  \
    if (f32_arith)                                                                               \
      return launch_cfg<a, b, cc, d, e, f, float, true>(s, vec, uf, ld, K, N, cst, gk, h, logD,  \
                                                        part, part_obj, part_flags, num_cus,     \
                                                        grid_out);                               \
    return f32 ? launch_cfg<a, b, cc, d, e, f>(s, vec, uf, ld, K, N, cst, gk, h, logD, part,     \
                                               part_obj, part_flags, num_cus, grid_out)          \
               : launch_cfg<a, b, cc, d, e, f>(s, vec, ud, ld, K, N, cst, gk, h, logD, part,     \
                                               part_obj, part_flags, num_cus, grid_out);         \
  }
  BUMBAR_CFG(4, 64, 2, 2, 1, 1)
  BUMBAR_CFG(4, 64, 2, 4, 1, 1)
  BUMBAR_CFG(4, 64, 2, 8, 1, 1)
  BUMBAR_CFG(4, 32, 2, 7, 1, 1)
  BUMBAR_CFG(4, 32, 2, 8, 1, 1)
  BUMBAR_CFG(4, 32, 2, 13, 0, 0)
  BUMBAR_CFG(4, 32, 2, 16, 0, 1)
  BUMBAR_CFG(8, 32, 2, 16, 0, 1)
#undef BUMBAR_CFG
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Robust two-pass sweep (any K; underflow-safe for arbitrarily poor f).
// ---------------------------------------------------------------------------

// Element (k, n) of u is at k * sk + n * sn: state-major (sk = ld, sn = 1) or
// the sample-major copy (sk = 1, sn = its row length).
// Pass A: exact ln D_n per column (thread per column).
template <typename TI>
__global__ void __launch_bounds__(256)
    robust_logD_kernel(const TI* __restrict__ u, int64_t sk, int64_t sn, int K, int64_t N,
                       const double* __restrict__ cst, const double* __restrict__ gk,
                       double* __restrict__ logD, unsigned* __restrict__ bad_out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned bad = 0;
  if (n < N) {
    double m = -INFINITY;
    for (int k = 0; k < K; ++k) {
      const double a = cst[k] - (double)u[(int64_t)k * sk + n * sn];
      if (gk[k] != 0.0) m = fmax(m, a);
      if (a != a || a == INFINITY) bad |= FLAG_NAN;
    }
    double D = 0.0;
    if (m > -INFINITY && m < INFINITY) {
      for (int k = 0; k < K; ++k)
        if (gk[k] != 0.0) D += exp_nonpos(cst[k] - (double)u[(int64_t)k * sk + n * sn] - m);
      logD[n] = m + log(D);
    } else {
      logD[n] = m;
      bad |= FLAG_COL;
    }
  }
  if (bad) atomicOr(bad_out, bad);
}

// Pass B: per-state online log-sum-exp of t_kn = ln h_n - u_kn - ln D_n over a
// chunk of columns; writes (M, S) with sum_{n in chunk} exp(t_kn) = S e^M, and
// the chunk's objective partial sum_n h_n ln D_n.
constexpr int kRobustThreads = 256;
constexpr int kRobustPerThread = 16;
constexpr int64_t kRobustChunk = (int64_t)kRobustThreads * kRobustPerThread;

int robust_chunks(int64_t N) { return (int)((N + kRobustChunk - 1) / kRobustChunk); }

__device__ __forceinline__ void lse_merge(double& m, double& s, double m2, double s2) {
  if (m2 == -INFINITY) return;
  if (m == -INFINITY) {
    m = m2;
    s = s2;
    return;
  }
  if (m2 > m) {
    s = s * exp_nonpos(m - m2) + s2;
    m = m2;
  } else {
    s = s + s2 * exp_nonpos(m2 - m);
  }
}

template <typename TI>
__global__ void __launch_bounds__(kRobustThreads)
    robust_state_kernel(const TI* __restrict__ u, int64_t sk, int64_t sn, int K, int64_t N,
                        const double* __restrict__ h, const double* __restrict__ logD,
                        double* __restrict__ partM, double* __restrict__ partS,
                        double* __restrict__ part_obj) {
  __shared__ double sm[kRobustThreads];
  __shared__ double ss[kRobustThreads];
  const int64_t base = (int64_t)blockIdx.x * kRobustChunk;
  const int tid = threadIdx.x;
  double lD[kRobustPerThread], lh[kRobustPerThread];
  double obj = 0.0;
#pragma unroll
  for (int i = 0; i < kRobustPerThread; ++i) {
    const int64_t n = base + tid + (int64_t)i * kRobustThreads;
    if (n < N) {
      lD[i] = logD[n];
      const double hn = h ? h[n] : 1.0;
      lh[i] = log(hn);
      obj += hn * lD[i];
    } else {
      lD[i] = INFINITY;
      lh[i] = -INFINITY;
    }
  }
  for (int k = 0; k < K; ++k) {
    double m = -INFINITY, s = 0.0;
#pragma unroll
    for (int i = 0; i < kRobustPerThread; ++i) {
      const int64_t n = base + tid + (int64_t)i * kRobustThreads;
      if (n < N) {
        const double t = lh[i] - (double)u[(int64_t)k * sk + n * sn] - lD[i];
        lse_merge(m, s, t, 1.0);
      }
    }
    sm[tid] = m;
    ss[tid] = s;
    __syncthreads();
    for (int w = kRobustThreads / 2; w > 0; w >>= 1) {
      if (tid < w) {
        double m1 = sm[tid], s1 = ss[tid];
        lse_merge(m1, s1, sm[tid + w], ss[tid + w]);
        sm[tid] = m1;
        ss[tid] = s1;
      }
      __syncthreads();
    }
    if (tid == 0) {
      partM[(int64_t)blockIdx.x * K + k] = sm[0];
      partS[(int64_t)blockIdx.x * K + k] = ss[0];
    }
    __syncthreads();
  }
  sm[tid] = obj;
  __syncthreads();
  for (int w = kRobustThreads / 2; w > 0; w >>= 1) {
    if (tid < w) sm[tid] += sm[tid + w];
    __syncthreads();
  }
  if (tid == 0) part_obj[blockIdx.x] = sm[0];
}

__global__ void zero_u32_kernel(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

template <typename TI>
static hipError_t launch_robust_t(hipStream_t s, const TI* u, int64_t sk, int64_t sn, int K,
                                  int64_t N,
                                  const double* cst, const double* gk, const double* h,
                                  double* logD, double* partM, double* partS, double* part_obj,
                                  unsigned* part_flags, int chunks) {
  hipLaunchKernelGGL(zero_u32_kernel, dim3((chunks + 255) / 256), dim3(256), 0, s, part_flags,
                     chunks);
  const int64_t nb = (N + 255) / 256;
  hipLaunchKernelGGL(robust_logD_kernel<TI>, dim3((unsigned)nb), dim3(256), 0, s, u, sk, sn, K, N,
                     cst, gk, logD, part_flags);
  hipLaunchKernelGGL(robust_state_kernel<TI>, dim3(chunks), dim3(kRobustThreads), 0, s, u, sk, sn,
                     K, N, h, logD, partM, partS, part_obj);
  return hipGetLastError();
}

hipError_t launch_sweep_robust(hipStream_t s, const void* u, bool f32, int64_t ld, int K, int64_t N,
                               const double* cst, const double* gk, const double* h,
                               double* logD, double* partM, double* partS, double* part_obj,
                               unsigned* part_flags, int chunks, bool sample_major) {
  // sample-major: ld is the row length of the copy
  const int64_t sk = sample_major ? 1 : ld, sn = sample_major ? ld : 1;
  if (f32)
    return launch_robust_t<float>(s, reinterpret_cast<const float*>(u), sk, sn, K, N, cst, gk, h,
                                  logD, partM, partS, part_obj, part_flags, chunks);
  return launch_robust_t<double>(s, reinterpret_cast<const double*>(u), sk, sn, K, N, cst, gk, h,
                                 logD, partM, partS, part_obj, part_flags, chunks);
}

// ---------------------------------------------------------------------------
// Finaliser: merges the workgroup partials in a fixed order and computes
// f_new, ln S, S, the gradient norm, Eq. (2) and flags. One workgroup of FT
// threads (256 for small problems, 1024 otherwise); the six scalar results
// are reduced together (wave butterflies, then the waves in order).
// ---------------------------------------------------------------------------
struct Red6 {
  double mdf, rs, gsq, minS, nf, ob;
};

template <int FT>
__device__ __forceinline__ Red6 block_reduce6(Red6 v, double (*sh)[6]) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    v.mdf = fmax(v.mdf, __shfl_xor(v.mdf, off, 64));
    v.rs = fmax(v.rs, __shfl_xor(v.rs, off, 64));
    v.gsq += __shfl_xor(v.gsq, off, 64);
    v.minS = fmin(v.minS, __shfl_xor(v.minS, off, 64));
    v.nf += __shfl_xor(v.nf, off, 64);
    v.ob += __shfl_xor(v.ob, off, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[w][0] = v.mdf;
    sh[w][1] = v.rs;
    sh[w][2] = v.gsq;
    sh[w][3] = v.minS;
    sh[w][4] = v.nf;
    sh[w][5] = v.ob;
  }
  __syncthreads();
  Red6 r{sh[0][0], sh[0][1], sh[0][2], sh[0][3], sh[0][4], sh[0][5]};
  for (int q = 1; q < FT / 64; ++q) {
    r.mdf = fmax(r.mdf, sh[q][0]);
    r.rs = fmax(r.rs, sh[q][1]);
    r.gsq += sh[q][2];
    r.minS = fmin(r.minS, sh[q][3]);
    r.nf += sh[q][4];
    r.ob += sh[q][5];
  }
  return r;
}

// Per-state sums of many state-major partials ahead of the finaliser: one
// wave per state, lane l adds partials l, l + 64, ... in eight chains (eight
// loads in flight per round trip), then a fixed xor butterfly, so the order
// of additions is fixed. S: K sums.
__global__ void __launch_bounds__(256)
    part_reduce_kernel(int K, int nparts, const double* __restrict__ part,
                       double* __restrict__ S) {
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= K) return;
  const double* pk = part + (int64_t)k * nparts;
  double s[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) s[j] = 0.0;
  int p = lane;
  for (; p + 7 * 64 < nparts; p += 8 * 64) {
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] += pk[p + 64 * j];
  }
  for (; p < nparts; p += 64) s[0] += pk[p];
  double v = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) S[k] = v;
}

// MODE 0: fast-path partials, 1: (M, S) pairs of the robust sweep.
// nstate: partials per state in part (mode 0: nparts, or 1 after
// part_reduce_kernel); nparts: entries of part_obj and part_flags.
template <int FT, int MODE>
__global__ void __launch_bounds__(FT)
    sweep_finalize_kernel(int K, int nstate, int nparts, const double* __restrict__ part,
                          const double* __restrict__ partS, const double* __restrict__ part_obj,
                          const unsigned* __restrict__ part_flags, const double* __restrict__ f,
                          const double* __restrict__ lnNp, const int64_t* __restrict__ Nk,
                          double* __restrict__ f_new, double* __restrict__ lnS_out,
                          double* __restrict__ S_out, SweepScalars* __restrict__ out,
                          double* __restrict__ cst_next) {
  __shared__ double sh[FT / 64][6];
  __shared__ double f0s;
  __shared__ unsigned flags_sh;
  // unnormalised f_new: in LDS when it fits (no global round trip before
  // the gauge is applied), else in f_new itself
  constexpr int kFinLds = 2048;
  __shared__ double fsh[kFinLds];
  double* fbuf = (K <= kFinLds) ? fsh : f_new;
  const int tid = threadIdx.x;
  if (tid == 0) flags_sh = 0u;
  // the first flag and objective partial of each thread are loaded up front,
  // together with the state partials below (one memory round trip, not three)
  const int t0 = tid < nparts ? tid : nparts - 1;
  const unsigned fl_first = part_flags[t0];
  const double ob_first = part_obj[t0];
  unsigned fl = tid < nparts ? fl_first : 0u;
  double ob0 = tid < nparts ? ob_first : 0.0;
  Red6 v{0.0, 0.0, 0.0, INFINITY, 0.0, 0.0};
  // Fast-path partials: T lanes per state (T a power of two, consecutive
  // lanes of one wave) each add every T-th partial, then a fixed xor
  // butterfly combines them, so the order of additions never changes.
  int T = 1;
  if (MODE == 0 && nstate > 1)
    while (T < 64 && 2 * T * K <= FT) T *= 2;
  const int kstride = FT / T;
  const int kfirst = tid / T, lane_c = tid % T;
  for (int k0 = 0; k0 < K; k0 += kstride) {
    const int k = k0 + kfirst;
    double Sp = 0.0;
    if (MODE == 0 && k < K) {
      // fast-path partials are state-major: part[k * nstate + p]
      // eight predicated loads in flight per lane, the ragged end included
      const double* pk = part + (int64_t)k * nstate;
      double a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = 0.0;
      // (clamped addresses and a select, not a branch per load: a branch
      // would wait for each load before the next)
      for (int p = lane_c; p < nstate; p += 8 * T) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int i = p + q * T;
          const double x = pk[i < nstate ? i : nstate - 1];
          a[q] += i < nstate ? x : 0.0;
        }
      }
#pragma unroll
      for (int w = 4; w >= 1; w >>= 1)
#pragma unroll
        for (int q = 0; q < w; ++q) a[q] += a[q + w];
      Sp = a[0];
    }
    if (MODE == 0)
      for (int off = 1; off < T; off <<= 1) Sp += __shfl_xor(Sp, off, 64);
    if (k >= K || lane_c != 0) continue;
    double lnS, fn, S;
    if (MODE == 0) {
      S = Sp;
      lnS = log(S);
      fn = lnNp[k] + f[k] - lnS;
      if (!(S >= 1e-290 && S <= 1e290)) fl |= FLAG_STATE;
    } else {
      double M = -INFINITY, Ssum = 0.0;
      for (int p = 0; p < nstate; ++p) lse_merge(M, Ssum, part[(int64_t)p * K + k],
                                                 partS[(int64_t)p * K + k]);
      const double lse = M + log(Ssum);  // ln sum_n h_n exp(-u_kn - ln D_n)
      fn = -lse;
      lnS = lnNp[k] + f[k] + lse;
      S = exp(lnS);
      if (!(lse > -INFINITY && lse < INFINITY)) fl |= FLAG_STATE;
    }
    if (lnS_out) lnS_out[k] = lnS;
    if (S_out) S_out[k] = S;
    fbuf[k] = fn;
    if (Nk[k] > 0) {
      const double g = S - (double)Nk[k];
      v.gsq += g * g;
      v.minS = fmin(v.minS, S);
    }
    if (fn != fn) fl |= FLAG_NAN;
  }
  for (int i = tid + FT; i < nparts; i += FT) {
    fl |= part_flags[i];
    ob0 += part_obj[i];
  }
  v.ob = ob0;
  __syncthreads();  // flags_sh initialised; f_new complete
  if (fl) atomicOr(&flags_sh, fl);
  if (tid == 0) f0s = fbuf[0];
  __syncthreads();
  const double f0 = f0s;
  for (int k = tid; k < K; k += FT) {
    const double fn = fbuf[k] - f0;
    f_new[k] = fn;
    // the constants of a sweep at f_new (what prepare_consts would write)
    if (cst_next) cst_next[k] = lnNp[k] + fn;
    double df = fabs(fn - f[k]);
    if (df != df) df = INFINITY;
    v.mdf = fmax(v.mdf, df);
    if (k >= 1) {
      double r;
      if (f[k] != 0.0)
        r = fabs(fn / f[k] - 1.0);
      else
        r = (fn == 0.0) ? 0.0 : INFINITY;
      if (r != r) r = INFINITY;
      v.rs = fmax(v.rs, r);
    }
    v.nf = __builtin_fma(-(double)Nk[k], f[k], v.nf);
  }
  const Red6 r = block_reduce6<FT>(v, sh);
  if (tid == 0) {
    out->max_df = r.mdf;
    out->rel_step = r.rs;
    out->objective = r.ob + r.nf;
    out->grad_norm = sqrt(r.gsq);
    out->min_S = r.minS;
    out->flags = flags_sh;
    out->pad = 0u;
  }
}

hipError_t launch_sweep_finalize(hipStream_t s, int mode, int K, int nparts, const double* part,
                                 double* partS, const double* part_obj,
                                 const unsigned* part_flags, const double* f, const double* lnNp,
                                 const int64_t* Nk, double* f_new, double* lnS, double* S_out,
                                 SweepScalars* out, double* cst_next) {
  // few partials: one wave-sized block; more: 1024 threads, with many
  // partials the per-state sums first, one wave per state over all CUs
  // (scratch: partS, which the fast-path mode does not use otherwise)
  if (K <= 256 && nparts <= 16) {
    if (mode == 0)
      hipLaunchKernelGGL((sweep_finalize_kernel<256, 0>), dim3(1), dim3(256), 0, s, K, nparts,
                         nparts, part, partS, part_obj, part_flags, f, lnNp, Nk, f_new, lnS, S_out,
                         out, cst_next);
    else
      hipLaunchKernelGGL((sweep_finalize_kernel<256, 1>), dim3(1), dim3(256), 0, s, K, nparts,
                         nparts, part, partS, part_obj, part_flags, f, lnNp, Nk, f_new, lnS, S_out,
                         out, cst_next);
    return hipGetLastError();
  }
  // the single workgroup takes about nparts / (8 T) dependent load rounds
  // (T lanes per state, as in the kernel); beyond a few rounds one more
  // launch that spreads the sums over the chip is cheaper
  int T = 1;
  while (T < 64 && 2 * T * K <= 1024) T *= 2;
  int nstate = nparts;
  if (mode == 0 && partS != nullptr && nparts > 32 * T) {
    hipLaunchKernelGGL(part_reduce_kernel, dim3((unsigned)((K + 3) / 4)), dim3(256), 0, s, K,
                       nparts, part, partS);
    part = partS;
    nstate = 1;
  }
  if (mode == 0)
    hipLaunchKernelGGL((sweep_finalize_kernel<1024, 0>), dim3(1), dim3(1024), 0, s, K, nstate,
                       nparts, part, partS, part_obj, part_flags, f, lnNp, Nk, f_new, lnS, S_out,
                       out, cst_next);
  else
    hipLaunchKernelGGL((sweep_finalize_kernel<1024, 1>), dim3(1), dim3(1024), 0, s, K, nstate,
                       nparts, part, partS, part_obj, part_flags, f, lnNp, Nk, f_new, lnS, S_out,
                       out, cst_next);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small kernels.
// ---------------------------------------------------------------------------
__global__ void prepare_consts_kernel(int K, const int64_t* __restrict__ Nk,
                                      const double* __restrict__ f, double* __restrict__ cst,
                                      double* __restrict__ gk, double* __restrict__ lnNp) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) {
    const double l = Nk[k] > 0 ? log((double)Nk[k]) : 0.0;
    lnNp[k] = l;
    cst[k] = l + f[k];
    gk[k] = Nk[k] > 0 ? 1.0 : 0.0;
  }
}

hipError_t launch_prepare_consts(hipStream_t s, int K, const int64_t* Nk, const double* f,
                                 double* cst, double* gk, double* lnNp) {
  hipLaunchKernelGGL(prepare_consts_kernel, dim3((K + 255) / 256), dim3(256), 0, s, K, Nk, f, cst,
                     gk, lnNp);
  return hipGetLastError();
}

__global__ void axpy_to_kernel(int K, const double* f, double alpha, const double* d, double* o) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < K) o[k] = __builtin_fma(alpha, d[k], f[k]);
}

hipError_t launch_axpy_to(hipStream_t s, int K, const double* f, double alpha, const double* d,
                          double* out) {
  hipLaunchKernelGGL(axpy_to_kernel, dim3((K + 255) / 256), dim3(256), 0, s, K, f, alpha, d, out);
  return hipGetLastError();
}

// Unsampled states: f_k <- f_k - ln S_k (= -ln sum_n exp(-u_kn - ln D_n), since
// ln N'_k = 0 for them), then the gauge f <- f - f_0. One block.
__global__ void __launch_bounds__(1024)
    fill_unsampled_gauge_kernel(int K, const int64_t* __restrict__ Nk, double* __restrict__ f,
                                const double* __restrict__ lnS) {
  __shared__ double f0;
  for (int k = threadIdx.x; k < K; k += blockDim.x)
    if (Nk[k] <= 0) f[k] = f[k] - lnS[k];
  __syncthreads();
  if (threadIdx.x == 0) f0 = f[0];
  __syncthreads();
  const double g = f0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) f[k] -= g;
}

hipError_t launch_fill_unsampled_gauge(hipStream_t s, int K, const int64_t* Nk, double* f,
                                       const double* lnS) {
  hipLaunchKernelGGL(fill_unsampled_gauge_kernel, dim3(1), dim3(1024), 0, s, K, Nk, f, lnS);
  return hipGetLastError();
}

__global__ void __launch_bounds__(1024)
    max_abs_diff_kernel(int K, const double* a, const double* b, double* out) {
  __shared__ double sh[1024];
  double m = 0.0;
  for (int k = threadIdx.x; k < K; k += 1024) {
    double d = fabs(a[k] - b[k]);
    if (d != d) d = INFINITY;
    m = fmax(m, d);
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

hipError_t launch_max_abs_diff(hipStream_t s, int K, const double* a, const double* b,
                               double* out) {
  hipLaunchKernelGGL(max_abs_diff_kernel, dim3(1), dim3(1024), 0, s, K, a, b, out);
  return hipGetLastError();
}

// W_nk = exp(f_k - u_kn - ln D_n), N x K output; 32 x 32 tiles transposed
// through shared memory so both the read of u (along n) and the write of W
// (along k) are coalesced.
template <typename TI>
__global__ void __launch_bounds__(256)
    weights_kernel(const TI* __restrict__ u, int64_t ld, int K, int64_t N,
                   const double* __restrict__ f, const double* __restrict__ logD,
                   double* __restrict__ W) {
  __shared__ double tile[32][33];
  const int64_t n0 = (int64_t)blockIdx.x * 32;
  const int k0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r;
    const int64_t n = n0 + tx;
    double v = 0.0;
    if (k < K && n < N) {
      const double x = f[k] - (double)u[(int64_t)k * ld + n] - logD[n];
      v = exp(x);
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t n = n0 + r;
    const int k = k0 + tx;
    if (k < K && n < N) W[n * K + k] = tile[tx][r];
  }
}

hipError_t launch_weights(hipStream_t s, const void* u, bool f32, int64_t ld, int K, int64_t N,
                          const double* f, const double* logD, double* W) {
  dim3 grid((unsigned)((N + 31) / 32), (unsigned)((K + 31) / 32));
  if (f32)
    hipLaunchKernelGGL(weights_kernel<float>, grid, dim3(256), 0, s,
                       reinterpret_cast<const float*>(u), ld, K, N, f, logD, W);
  else
    hipLaunchKernelGGL(weights_kernel<double>, grid, dim3(256), 0, s,
                       reinterpret_cast<const double*>(u), ld, K, N, f, logD, W);
  return hipGetLastError();
}

// Reweighting (Eqs. (5)-(6)): p_n = exp(t_n - M) / sum_m exp(t_m - M),
// t_n = -u_target_n - ln D_n. Three launches: block maxima, one block
// merging (M, S) in a fixed order, then the normalised write.
__global__ void __launch_bounds__(256)
    rw_partial_kernel(int64_t N, const double* __restrict__ ut, const double* __restrict__ logD,
                      double* __restrict__ part) {
  __shared__ double sm[256], ss[256];
  double m = -INFINITY, s = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < N; n += (int64_t)gridDim.x * 256)
    lse_merge(m, s, -ut[n] - logD[n], 1.0);
  sm[threadIdx.x] = m;
  ss[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      double m1 = sm[threadIdx.x], s1 = ss[threadIdx.x];
      lse_merge(m1, s1, sm[threadIdx.x + w], ss[threadIdx.x + w]);
      sm[threadIdx.x] = m1;
      ss[threadIdx.x] = s1;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sm[0];
    part[2 * blockIdx.x + 1] = ss[0];
  }
}

__global__ void rw_merge_kernel(int nparts, double* part) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double m = -INFINITY, s = 0.0;
    for (int p = 0; p < nparts; ++p) lse_merge(m, s, part[2 * p], part[2 * p + 1]);
    part[2 * nparts] = m + log(s);
  }
}

__global__ void rw_write_kernel(int64_t N, const double* __restrict__ ut,
                                const double* __restrict__ logD, const double* __restrict__ lse,
                                double* __restrict__ p) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N) p[n] = exp(-ut[n] - logD[n] - *lse);
}

hipError_t launch_reweight(hipStream_t s, int64_t N, const double* ut, const double* logD,
                           double* part, int nparts, double* p) {
  hipLaunchKernelGGL(rw_partial_kernel, dim3(nparts), dim3(256), 0, s, N, ut, logD, part);
  hipLaunchKernelGGL(rw_merge_kernel, dim3(1), dim3(64), 0, s, nparts, part);
  hipLaunchKernelGGL(rw_write_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, ut,
                     logD, part + 2 * nparts, p);
  return hipGetLastError();
}

__global__ void check_finite_kernel(int K, const double* f, unsigned* flag) {
  unsigned bad = 0;
  for (int k = threadIdx.x; k < K; k += blockDim.x)
    if (!(f[k] > -INFINITY && f[k] < INFINITY)) bad = 1;
  if (bad) atomicOr(flag, 1u);
}

hipError_t launch_check_finite_f(hipStream_t s, int K, const double* f, unsigned* flag) {
  hipLaunchKernelGGL(check_finite_kernel, dim3(1), dim3(256), 0, s, K, f, flag);
  return hipGetLastError();
}

}  // namespace bumbar
