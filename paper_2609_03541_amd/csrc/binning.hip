// Binning on the GPU (Section 2, text after Eq. (1)): quantisation of the
// sampled coordinates, the nonempty-bin count g(m) for a width of m quanta,
// the histogram over the nonempty bins and the bin representatives.
//
// Everything after quantisation is integer arithmetic, so the bins, counts
// and the width found by the bisection are bit-identical to any correct
// implementation of the same definitions. g(m) is computed from sorted keys
// (distinct values are the run starts of a sorted sequence) in 1-D, where the
// quantised coordinates are sorted once because q -> q / m is monotone, so
// every probe is a single pass over N integers; in 2-D the row-major cell id
// is not monotone in (q_y, q_x) for all m, so a probe marks the occupied
// cells in a bitmap (LDS-privatised, integer atomics) and counts its bits,
// or, for grids too large for the bitmap, sorts the cell ids. The histogram
// takes the run starts and run lengths of the sorted cell ids.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "bumbar_impl.h"
#include "solver_internal.h"

namespace bumbar {

constexpr int kBT = 256;
constexpr int kRedBlocks = 1024;

// ---- min / max per dimension --------------------------------------------
__global__ void __launch_bounds__(kBT)
    minmax_partial_kernel(const double* __restrict__ xi, int64_t N, int d,
                          double* __restrict__ part) {
  __shared__ double smin[kBT], smax[kBT];
  for (int j = 0; j < d; ++j) {
    double a = INFINITY, b = -INFINITY;
    for (int64_t n = (int64_t)blockIdx.x * kBT + threadIdx.x; n < N;
         n += (int64_t)gridDim.x * kBT) {
      const double v = xi[n * d + j];
      a = fmin(a, v);
      b = fmax(b, v);
      if (v != v) {
        a = -INFINITY;  // poison: reported as non-finite
        b = INFINITY;
      }
    }
    smin[threadIdx.x] = a;
    smax[threadIdx.x] = b;
    __syncthreads();
    for (int w = kBT / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
        smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      part[(blockIdx.x * 2 + 0) * 2 + j] = smin[0];
      part[(blockIdx.x * 2 + 1) * 2 + j] = smax[0];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBT)
    minmax_final_kernel(int nparts, int d, const double* __restrict__ part,
                        double* __restrict__ mm) {
  __shared__ double smin[kBT], smax[kBT];
  for (int j = 0; j < d; ++j) {
    double a = INFINITY, b = -INFINITY;
    for (int p = threadIdx.x; p < nparts; p += kBT) {
      a = fmin(a, part[(p * 2 + 0) * 2 + j]);
      b = fmax(b, part[(p * 2 + 1) * 2 + j]);
    }
    smin[threadIdx.x] = a;
    smax[threadIdx.x] = b;
    __syncthreads();
    for (int w = kBT / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) {
        smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
        smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      mm[2 * j] = smin[0];
      mm[2 * j + 1] = smax[0];
    }
    __syncthreads();
  }
}

hipError_t launch_minmax(hipStream_t s, const double* xi, int64_t N, int d, double* mm,
                         int64_t* scratch) {
  double* part = reinterpret_cast<double*>(scratch);
  int nb = (int)std::min<int64_t>(kRedBlocks, (N + kBT - 1) / kBT);
  hipLaunchKernelGGL(minmax_partial_kernel, dim3(nb), dim3(kBT), 0, s, xi, N, d, part);
  hipLaunchKernelGGL(minmax_final_kernel, dim3(1), dim3(kBT), 0, s, nb, d, part, mm);
  return hipGetLastError();
}

// ---- quantisation ---------------------------------------------------------
// lo = min, scale = (2^32 - 1) / (max - min) (0 if max = min),
// q = min(floor((x - lo) * scale), 2^32 - 1); separate IEEE subtract and
// multiply (no contraction is possible for (x - lo) * scale).
__global__ void quantize_params_kernel(int d, const double* __restrict__ mm, double* lo,
                                       double* scale, unsigned* bad) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    unsigned b = 0;
    for (int j = 0; j < d; ++j) {
      const double a = mm[2 * j], c = mm[2 * j + 1];
      if (!(a > -INFINITY && c < INFINITY)) b = 1;
      lo[j] = a;
      scale[j] = (c > a) ? 4294967295.0 / (c - a) : 0.0;
    }
    *bad = b;
  }
}

__global__ void __launch_bounds__(kBT)
    quantize_kernel(const double* __restrict__ xi, int64_t N, int d,
                    const double* __restrict__ lo, const double* __restrict__ scale,
                    uint32_t* __restrict__ q) {
  const int64_t e = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (e >= N * d) return;
  const int j = (int)(e % d);
  const double diff = __dsub_rn(xi[e], lo[j]);
  double fl = floor(__dmul_rn(diff, scale[j]));
  if (fl > 4294967295.0) fl = 4294967295.0;
  if (!(fl >= 0.0)) fl = 0.0;
  q[e] = (uint32_t)fl;
}

hipError_t launch_quantize(hipStream_t s, const double* xi, int64_t N, int d, const double* mm,
                           double* lo, double* scale, uint32_t* q, unsigned* bad) {
  hipLaunchKernelGGL(quantize_params_kernel, dim3(1), dim3(64), 0, s, d, mm, lo, scale, bad);
  const int64_t tot = N * d;
  hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)((tot + kBT - 1) / kBT)), dim3(kBT), 0, s, xi,
                     N, d, lo, scale, q);
  return hipGetLastError();
}

// ---- sorting ----------------------------------------------------------------
__global__ void iota_kernel(uint32_t* p, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (i < N) p[i] = (uint32_t)i;
}

size_t sort_temp_bytes(int64_t N) {
  return std::max(radix_temp_bytes(N), scan_temp_bytes(N)) + 1024;
}

hipError_t launch_sort_1d(hipStream_t s, const uint32_t* q, int64_t N, uint32_t* iota,
                          uint32_t* q_sorted, uint32_t* perm, void* tmp, size_t tmp_bytes) {
  hipLaunchKernelGGL(iota_kernel, dim3((unsigned)((N + kBT - 1) / kBT)), dim3(kBT), 0, s, iota,
                     N);
  return radix_sort_u32(s, q, q_sorted, iota, perm, N, 32, tmp, tmp_bytes);
}

// ---- distinct counting -----------------------------------------------------
// counts[1 + b] = number of run starts in block b's range; counts[0] = total.
__global__ void __launch_bounds__(kBT)
    count_runs_1d_kernel(const uint32_t* __restrict__ qs, int64_t N, uint64_t m,
                         int64_t* __restrict__ counts) {
  __shared__ int64_t sh[kBT];
  int64_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBT) {
    const uint64_t a = (uint64_t)qs[i] / m;
    c += (i == 0) ? 1 : (a != (uint64_t)qs[i - 1] / m);
  }
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int w = kBT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[1 + blockIdx.x] = sh[0];
}

template <typename TK>
__global__ void __launch_bounds__(kBT)
    count_runs_keys_kernel(const TK* __restrict__ ks, int64_t N, int64_t* __restrict__ counts) {
  __shared__ int64_t sh[kBT];
  int64_t c = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBT)
    c += (i == 0) ? 1 : (ks[i] != ks[i - 1]);
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int w = kBT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[1 + blockIdx.x] = sh[0];
}

// counts[0] = sum of the nb block counts (integer, so the order is irrelevant).
__global__ void __launch_bounds__(kBT) sum_counts_kernel(int nb, int64_t* counts) {
  __shared__ int64_t sh[kBT];
  int64_t t = 0;
  for (int b = threadIdx.x; b < nb; b += kBT) t += counts[1 + b];
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int w = kBT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[0] = sh[0];
}

// g(m) for up to kMaxProbes widths in one pass over the sorted coordinates:
// counts[j] = number of distinct floor(q / m_j) (run starts, integer atomics,
// so the totals do not depend on the order of the additions).
//
// The divisions use a multiplier per width: for 2 <= m < 2^32 and q < 2^32,
// floor(q / m) = floor(q * M / 2^64) exactly with M = ceil(2^64 / m) (the
// error q (M m - 2^64) / (m 2^64) stays below 2^-32 < 1/m, so it never
// crosses an integer); m = 1 gives q, and m >= 2^32 gives 0.
constexpr int kMaxProbes = 64;

__device__ __forceinline__ uint32_t div_by_magic(uint32_t q, uint64_t m, uint64_t magic) {
  if (m == 1) return q;
  if (m > 0xffffffffull) return 0u;
  const uint32_t lo = (uint32_t)magic, hi = (uint32_t)(magic >> 32);
  const uint64_t t = (uint64_t)q * hi + __umulhi(q, lo);
  return (uint32_t)(t >> 32);
}

constexpr int kRunChunk = 256;  // sorted coordinates per wave and pass

// Lane (p, s) of a wave counts, for width m_p, the positions where
// floor(q / m_p) changes (one division per element, against the previous
// element's) in stream s of a chunk of kRunChunk consecutive sorted
// coordinates. With MP probe slots (a power of two >= the number of probes)
// a chunk splits into 64 / MP streams, so a pass costs N x MP lane steps:
// with all 64 slots every lane reads the same coordinate at a time. Nothing
// is exchanged between lanes until one sum per block and probe, added with
// one integer atomic.
__global__ void __launch_bounds__(kBT)
    count_runs_1d_multi_kernel(const uint32_t* __restrict__ qs, int64_t N,
                               const WidthSearch1D* __restrict__ ws, int MP) {
  __shared__ unsigned long long sred[kBT / 64][kMaxProbes];
  const int M = ws->M;  // 0 once the search has ended: nothing to count
  if (M == 0) return;
  const uint64_t* ms = ws->ms;
  unsigned long long* counts = const_cast<WidthSearch1D*>(ws)->counts;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int p = lane % MP, st = lane / MP;
  const int len = kRunChunk / (64 / MP);  // coordinates per stream
  const bool act = p < M;
  const uint64_t m = act ? ms[2 * p] : 1ull;
  const uint64_t mg = act ? ms[2 * p + 1] : 0ull;
  const int64_t nchunks = (N + kRunChunk - 1) / kRunChunk;
  const int64_t nw = (int64_t)gridDim.x * (kBT / 64);
  unsigned long long c = 0;
  for (int64_t ch = (int64_t)blockIdx.x * (kBT / 64) + wave; ch < nchunks; ch += nw) {
    const int64_t b = ch * kRunChunk + (int64_t)st * len;
    const int64_t e = std::min<int64_t>(N, b + len);
    if (b >= e) continue;
    int64_t i = b;
    uint32_t dp;
    if (b == 0) {
      dp = div_by_magic(qs[0], m, mg);
      c += 1;  // the first coordinate starts a run
      i = 1;
    } else {
      dp = div_by_magic(qs[b - 1], m, mg);
    }
#pragma unroll 8
    for (; i < e; ++i) {
      const uint32_t d = div_by_magic(qs[i], m, mg);
      c += d != dp ? 1ull : 0ull;
      dp = d;
    }
  }
  sred[wave][lane] = c;
  __syncthreads();
  if (threadIdx.x < M) {
    unsigned long long t = 0;
    for (int w = 0; w < kBT / 64; ++w)
      for (int q = 0; q < 64 / MP; ++q) t += sred[w][q * MP + threadIdx.x];
    if (t) atomicAdd(&counts[threadIdx.x], t);
  }
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

static int red_blocks(int64_t N) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(kRedBlocks, (N + kBT - 1) / kBT));
}

hipError_t launch_count_1d(hipStream_t s, const uint32_t* q_sorted, int64_t N, uint64_t m,
                           int64_t* counts) {
  const int nb = red_blocks(N);
  hipLaunchKernelGGL(count_runs_1d_kernel, dim3(nb), dim3(kBT), 0, s, q_sorted, N, m, counts);
  hipLaunchKernelGGL(sum_counts_kernel, dim3(1), dim3(kBT), 0, s, nb, counts);
  return hipGetLastError();
}

__host__ __device__ static uint64_t magic_of(uint64_t m) {
  if (m < 2 || m > 0xffffffffull) return 0;
  return ~0ull / m + 1ull;  // ceil(2^64 / m)
}

// Appends to nm (LDS) the midpoints of the next `levels` levels of the
// bisection tree under (lo, hi): the interval at depth d along the path code
// c (bit i: right half at step i) has its midpoint probed if it is wider
// than one. Single thread; returns the new count.
__device__ static int ws_emit(uint64_t lo, uint64_t hi, int levels, uint64_t* nm, int M) {
  for (int d = 0; d < levels; ++d) {
    for (int c = 0; c < (1 << d); ++c) {
      uint64_t a = lo, b = hi;
      bool ok = true;
      for (int i = 0; i < d; ++i) {
        if (b - a <= 1) {
          ok = false;
          break;
        }
        const uint64_t mid = a + (b - a) / 2;
        if ((c >> i) & 1)
          a = mid;
        else
          b = mid;
      }
      if (!ok || b - a <= 1) continue;
      nm[M++] = a + (b - a) / 2;
    }
  }
  return M;
}

// Writes the probes of the next pass (m and its magic number, counts zeroed)
// with every thread of the block; nm and M in LDS.
__device__ static void ws_store(WidthSearch1D* w, const uint64_t* nm, int M) {
  for (int t = threadIdx.x; t < M; t += blockDim.x) {
    w->ms[2 * t] = nm[t];
    w->ms[2 * t + 1] = magic_of(nm[t]);
    w->counts[t] = 0ull;
  }
}

// First pass: m = 1 and the midpoints of the top `levels` levels.
__global__ void __launch_bounds__(64) ws_init_kernel(WidthSearch1D* w, int64_t n, int levels) {
  __shared__ uint64_t nm[kMaxProbes];
  __shared__ int sM;
  if (threadIdx.x == 0) {
    nm[0] = 1;
    sM = ws_emit(1, 4294967296ull, levels, nm, 1);
    w->lo = 1;
    w->hi = 4294967296ull;
    w->glo = 0;
    w->n = n;
    w->levels = levels;
    w->done = 0;
    w->first = 1;
    w->M = sM;
  }
  __syncthreads();
  ws_store(w, nm, sM);
}

// Walks the evaluated part of the tree exactly as the bisection would, then
// queues the next pass (or ends the search: M = 0, done = 1). The probes and
// their counts are staged in LDS by the whole block; one thread walks.
__global__ void __launch_bounds__(64) ws_walk_kernel(WidthSearch1D* w) {
  __shared__ uint64_t sm[kMaxProbes];
  __shared__ unsigned long long sc[kMaxProbes];
  __shared__ uint64_t nm[kMaxProbes];
  __shared__ int sM;
  if (w->done) return;  // uniform: every thread reads the same flag
  const int M = w->M;
  for (int t = threadIdx.x; t < M; t += blockDim.x) {
    sm[t] = w->ms[2 * t];
    sc[t] = w->counts[t];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sM = 0;
    const int64_t n = w->n;
    uint64_t lo = w->lo, hi = w->hi;
    int64_t glo = w->glo;
    bool finished = false;
    if (w->first) {
      const int64_t g1 = (int64_t)sc[0];
      w->first = 0;
      if (g1 < n) {  // even the finest width gives fewer than n bins
        lo = 1;
        glo = g1;
        finished = true;
      } else {
        glo = g1;
      }
    }
    while (!finished && hi - lo > 1) {
      const uint64_t mid = lo + (hi - lo) / 2;
      int j = -1;
      for (int q = 0; q < M; ++q)
        if (sm[q] == mid) {
          j = q;
          break;
        }
      if (j < 0) break;  // outside this pass's subtree
      const int64_t gm = (int64_t)sc[j];
      if (gm >= n) {
        lo = mid;
        glo = gm;
      } else {
        hi = mid;
      }
    }
    if (hi - lo <= 1) finished = true;
    w->lo = lo;
    w->hi = hi;
    w->glo = glo;
    if (!finished) sM = ws_emit(lo, hi, w->levels, nm, 0);
    w->M = sM;
    w->done = finished ? 1 : 0;
  }
  __syncthreads();
  ws_store(w, nm, sM);
}

// The whole bisection in one workgroup, for N <= kWsSmallN: thread t keeps
// the kWsL sorted coordinates from t kWsL on in registers (and the one
// before them), and each probe is a count of run starts over them plus a
// workgroup sum. g(1) first; if g(1) < n the width is 1, else the interval
// [1, 2^32] is halved until hi - lo = 1, keeping g(lo) >= n, as the
// multi-pass search does. Ends the search (done = 1) in w.
constexpr int kWsT = 1024;
constexpr int kWsL = 16;
constexpr int64_t kWsSmallN = (int64_t)kWsT * kWsL;

__global__ void __launch_bounds__(kWsT)
    ws_small_kernel(const uint32_t* __restrict__ qs, int64_t N, int64_t n, WidthSearch1D* w) {
  __shared__ unsigned part[kWsT / 64];
  __shared__ unsigned total;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int64_t b = (int64_t)t * kWsL;
  uint32_t q[kWsL];
#pragma unroll
  for (int j = 0; j < kWsL; ++j) q[j] = b + j < N ? qs[b + j] : 0u;
  const uint32_t before = (b > 0 && b < N) ? qs[b - 1] : 0u;
  auto count = [&](uint64_t m) -> int64_t {
    const uint64_t mg = magic_of(m);
    uint32_t dp = div_by_magic(before, m, mg);
    unsigned c = 0u;
#pragma unroll
    for (int j = 0; j < kWsL; ++j) {
      if (b + j < N) {
        const uint32_t d = div_by_magic(q[j], m, mg);
        c += (b + j == 0) ? 1u : (d != dp ? 1u : 0u);
        dp = d;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane == 0) part[wave] = c;
    __syncthreads();
    if (t == 0) {
      unsigned a = 0u;
      for (int v = 0; v < kWsT / 64; ++v) a += part[v];
      total = a;
    }
    __syncthreads();
    return (int64_t)total;
  };
  uint64_t lo = 1, hi = 4294967296ull;
  int64_t glo = count(1);
  if (glo >= n) {
    while (hi - lo > 1) {
      const uint64_t mid = lo + (hi - lo) / 2;
      const int64_t gm = count(mid);
      if (gm >= n) {
        lo = mid;
        glo = gm;
      } else {
        hi = mid;
      }
    }
  }
  if (t == 0) {
    w->lo = lo;
    w->hi = hi;
    w->glo = glo;
    w->n = n;
    w->levels = 0;
    w->M = 0;
    w->done = 1;
    w->first = 0;
  }
}

hipError_t launch_width_search_1d(hipStream_t s, const uint32_t* q_sorted, int64_t N,
                                  int64_t n, int levels, int passes, bool init,
                                  WidthSearch1D* w) {
  if (levels < 1 || levels > 6 || passes < 1) return hipErrorInvalidValue;
  if (init && N <= kWsSmallN) {
    hipLaunchKernelGGL(ws_small_kernel, dim3(1), dim3(kWsT), 0, s, q_sorted, N, n, w);
    return hipGetLastError();
  }
  int MP = 4;  // probe slots per wave: a power of two, 64 / MP streams of >= 4 coordinates
  while (MP < (1 << levels)) MP *= 2;
  const int64_t nchunks = (N + kRunChunk - 1) / kRunChunk;
  const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(1024, (nchunks + 3) / 4));
  if (init) hipLaunchKernelGGL(ws_init_kernel, dim3(1), dim3(64), 0, s, w, n, levels);
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(count_runs_1d_multi_kernel, dim3((unsigned)nb), dim3(kBT), 0, s, q_sorted,
                       N, w, MP);
    hipLaunchKernelGGL(ws_walk_kernel, dim3(1), dim3(64), 0, s, w);
  }
  return hipGetLastError();
}

// 2-D row-major cell id with the first coordinate fastest:
//   c = q0 / m + (q1 / m) * (floor((2^32 - 1) / m) + 1)
__device__ __forceinline__ uint64_t cell2(uint32_t q0, uint32_t q1, uint64_t m) {
  const uint64_t stride = 4294967295ull / m + 1ull;
  return (uint64_t)q0 / m + ((uint64_t)q1 / m) * stride;
}

__global__ void cells_kernel(const uint32_t* __restrict__ q, int64_t N, int d, uint64_t m,
                             uint64_t* __restrict__ keys) {
  const int64_t n = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (n >= N) return;
  keys[n] = (d == 1) ? (uint64_t)q[n] / m : cell2(q[2 * n], q[2 * n + 1], m);
}

// The same 2-D cell ids when every id of this m fits in 32 bits.
__global__ void cells32_kernel(const uint32_t* __restrict__ q, int64_t N, uint64_t m,
                               uint32_t* __restrict__ keys) {
  const int64_t n = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (n >= N) return;
  keys[n] = (uint32_t)cell2(q[2 * n], q[2 * n + 1], m);
}

static unsigned key_bits(int d, uint64_t m) {
  // the largest possible cell id for this m, then its bit length
  uint64_t maxc;
  if (d == 1) {
    maxc = 4294967295ull / m;
  } else {
    const uint64_t stride = 4294967295ull / m + 1ull;
    maxc = (4294967295ull / m) + (4294967295ull / m) * stride;
  }
  unsigned b = 1;
  while (b < 64 && (maxc >> b) != 0) ++b;
  return b;
}

// ---- 2-D g(m) as an occupancy histogram ------------------------------------
// The cells of width m form an ncx x ncx grid (ncx = floor((2^32 - 1) / m) +
// 1, row-major ids as cell2). g(m) is the number of occupied cells: each
// sample sets its cell's bit in a bitmap of the grid with an integer atomic
// OR, then the set bits are counted. Small grids (the coarse widths at the
// start of the bisection, where many samples share few cells) are marked in
// a bitmap private to each workgroup in LDS and merged into the global one
// word by word; larger grids are marked in the global bitmap directly (few
// samples per cell, little contention). Integer operations only, so the count
// is exact and does not depend on the order of the atomics.
constexpr int kLdsWords = 8192;  // 32 KB of LDS: grids of up to 262144 cells

__global__ void __launch_bounds__(kBT) zero_words_kernel(uint32_t* w, int64_t nw) {
  for (int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x; i < nw; i += (int64_t)gridDim.x * kBT)
    w[i] = 0u;
}

__global__ void __launch_bounds__(kBT)
    mark_cells_kernel(const uint32_t* __restrict__ q, int64_t N, uint64_t m, uint64_t magic,
                      uint64_t ncx, int64_t nw, uint32_t* __restrict__ words) {
  __shared__ uint32_t lw[kLdsWords];
  const bool private_map = nw <= kLdsWords;  // uniform over the grid
  if (private_map) {
    for (int i = threadIdx.x; i < nw; i += kBT) lw[i] = 0u;
    __syncthreads();
  }
  for (int64_t n = (int64_t)blockIdx.x * kBT + threadIdx.x; n < N; n += (int64_t)gridDim.x * kBT) {
    const uint64_t c = (uint64_t)div_by_magic(q[2 * n], m, magic) +
                       (uint64_t)div_by_magic(q[2 * n + 1], m, magic) * ncx;
    const uint32_t bit = 1u << (uint32_t)(c & 31u);
    // bits are only ever set: a bit seen set is set, so its atomic is
    // skipped (most samples land in cells already marked); a stale read only
    // costs a redundant atomic
    if (private_map) {
      if (!(lw[c >> 5] & bit)) atomicOr(&lw[c >> 5], bit);
    } else {
      if (!(words[c >> 5] & bit)) atomicOr(&words[c >> 5], bit);
    }
  }
  if (private_map) {
    __syncthreads();
    for (int i = threadIdx.x; i < nw; i += kBT)
      if (lw[i]) atomicOr(&words[i], lw[i]);
  }
}

// counts[0] += number of set bits (per-block sums, one integer atomic each)
__global__ void __launch_bounds__(kBT)
    popcount_words_kernel(const uint32_t* __restrict__ w, int64_t nw,
                          unsigned long long* __restrict__ total) {
  __shared__ unsigned long long sh[kBT];
  unsigned long long c = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x; i < nw; i += (int64_t)gridDim.x * kBT)
    c += (unsigned long long)__builtin_popcount(w[i]);
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int s2 = kBT / 2; s2 > 0; s2 >>= 1) {
    if (threadIdx.x < s2) sh[threadIdx.x] += sh[threadIdx.x + s2];
    __syncthreads();
  }
  if (threadIdx.x == 0 && sh[0]) atomicAdd(total, sh[0]);
}

// Bits of the occupancy bitmap of width m (0 if its grid is beyond 2^62 cells).
static uint64_t grid_cells_2d(uint64_t m) {
  const uint64_t ncx = 4294967295ull / m + 1ull;
  if (ncx > (1ull << 31)) return 0;
  return ncx * ncx;
}

static bool count_2d_uses_bitmap(int64_t N, uint64_t m) {
  const uint64_t g = grid_cells_2d(m);
  // the bitmap lives in the N x 8 bytes of the key buffer
  return g != 0 && g <= (uint64_t)N * 64ull;
}

// ---- 2-D width search on the device ------------------------------------
//
// The bisection of the host loop, one probe per pass, with every probe whose
// grid fits the bitmap run on the device: zero the bitmap, mark the cells,
// count the bits, and a one-thread walk takes the bisection step and prepares
// the next probe (or ends the search, or hands it back to the host when the
// next grid is too large for the bitmap). The passes are queued back to back;
// the host reads the state once at the end.
__device__ static void ws2_prepare(WidthSearch2D* w) {
  const uint64_t mid = w->lo + (w->hi - w->lo) / 2;
  const uint64_t ncx = 4294967295ull / mid + 1ull;
  const bool fits = ncx <= (1ull << 31) && ncx * ncx <= w->cap_cells;
  if (!fits) {
    w->host = 1;
    return;
  }
  w->m = mid;
  w->magic = magic_of(mid);
  w->ncx = ncx;
  w->nw = (int64_t)((ncx * ncx + 31) / 32);
  w->count = 0ull;
}

__global__ void ws2_init_kernel(WidthSearch2D* w, int64_t n, int64_t g1, uint64_t cap_cells) {
  w->lo = 1;
  w->hi = 4294967296ull;
  w->glo = g1;
  w->n = n;
  w->cap_cells = cap_cells;
  w->done = 0;
  w->host = 0;
  ws2_prepare(w);
}

__global__ void __launch_bounds__(kBT) ws2_zero_kernel(const WidthSearch2D* w, uint32_t* words) {
  if (w->done || w->host) return;  // uniform
  const int64_t nw = w->nw;
  for (int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x; i < nw; i += (int64_t)gridDim.x * kBT)
    words[i] = 0u;
}

// One probe over the samples sorted by (q_y, q_x) (key q_y 2^32 + q_x):
// workgroup b takes the run [b L, (b + 1) L). Sorted by q_y, its cells lie in
// the rows q_y / m of its first to its last sample, one contiguous range of
// ids, which is marked in an LDS window when it fits (the whole grid at
// coarse widths, a band of a few rows at fine ones) and OR-ed into the global
// bitmap word by word; otherwise the global bitmap is marked directly. Each
// workgroup counts the bits it is the first to set (the word an atomic OR
// returns shows which were set before), so w->count ends as the number of
// occupied cells whatever the order of the atomics.
__global__ void __launch_bounds__(kBT)
    ws2_mark_kernel(const uint64_t* __restrict__ qs, int64_t N, int64_t L,
                    WidthSearch2D* w, uint32_t* __restrict__ words) {
  if (w->done || w->host) return;  // uniform
  __shared__ uint32_t lw[kLdsWords];
  __shared__ unsigned long long sh[kBT / 64];
  const uint64_t m = w->m, magic = w->magic, ncx = w->ncx;
  const int64_t n0 = (int64_t)blockIdx.x * L;
  const int64_t n1 = n0 + L < N ? n0 + L : N;
  if (n0 >= n1) return;  // uniform
  const uint64_t w_lo = (uint64_t)div_by_magic((uint32_t)(qs[n0] >> 32), m, magic) * ncx >> 5;
  const uint64_t w_hi =
      ((uint64_t)div_by_magic((uint32_t)(qs[n1 - 1] >> 32), m, magic) * ncx + ncx - 1) >> 5;
  const int64_t nwin = (int64_t)(w_hi - w_lo) + 1;
  const bool window = nwin <= kLdsWords;  // uniform over the workgroup
  unsigned long long fresh = 0;
  if (window) {
    for (int i = threadIdx.x; i < nwin; i += kBT) lw[i] = 0u;
    __syncthreads();
  }
  for (int64_t n = n0 + threadIdx.x; n < n1; n += kBT) {
    const uint64_t key = qs[n];
    const uint64_t c = (uint64_t)div_by_magic((uint32_t)key, m, magic) +
                       (uint64_t)div_by_magic((uint32_t)(key >> 32), m, magic) * ncx;
    const uint32_t bit = 1u << (uint32_t)(c & 31u);
    // bits are only ever set: a bit seen set is set, so its atomic is
    // skipped (most samples land in cells already marked)
    if (window) {
      uint32_t* wp = &lw[(c >> 5) - w_lo];
      if (!(*wp & bit)) atomicOr(wp, bit);
    } else {
      uint32_t* wp = &words[c >> 5];
      if (!(*wp & bit) && !(atomicOr(wp, bit) & bit)) ++fresh;
    }
  }
  if (window) {
    __syncthreads();
    for (int64_t i = threadIdx.x; i < nwin; i += kBT) {
      const uint32_t v = lw[i];
      if (v) fresh += (unsigned long long)__builtin_popcount(v & ~atomicOr(&words[w_lo + i], v));
    }
  }
  for (int off = 32; off > 0; off >>= 1) fresh += __shfl_xor(fresh, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = fresh;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int i = 0; i < kBT / 64; ++i) t += sh[i];
    if (t) atomicAdd(&w->count, t);
  }
}

__global__ void ws2_walk_kernel(WidthSearch2D* w) {
  if (w->done || w->host) return;
  const int64_t gm = (int64_t)w->count;
  if (gm >= w->n) {
    w->lo = w->m;
    w->glo = gm;
  } else {
    w->hi = w->m;
  }
  if (w->hi - w->lo <= 1) {
    w->done = 1;
    return;
  }
  ws2_prepare(w);
}

// samples per workgroup of the sorted probe: at least 8 per thread, at most
// 2048 workgroups
static int64_t ws2_run(int64_t N) {
  const int64_t by_grid = (N + 2047) / 2048;
  return by_grid > 8 * kBT ? by_grid : 8 * kBT;
}

hipError_t launch_width_search_2d(hipStream_t s, const uint64_t* qs, int64_t N, int64_t n,
                                  int64_t g1, int passes, bool init, uint64_t* bitmap,
                                  WidthSearch2D* w) {
  if (passes < 1) return hipErrorInvalidValue;
  // the bitmap lives in N x 8 bytes: at most 64 N cells
  if (init) hipLaunchKernelGGL(ws2_init_kernel, dim3(1), dim3(1), 0, s, w, n, g1, (uint64_t)N * 64ull);
  uint32_t* words = reinterpret_cast<uint32_t*>(bitmap);
  const unsigned zb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (2 * N + kBT - 1) / kBT));
  const int64_t L = ws2_run(N);
  const unsigned mb = (unsigned)((N + L - 1) / L);
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(ws2_zero_kernel, dim3(zb), dim3(kBT), 0, s, w, words);
    hipLaunchKernelGGL(ws2_mark_kernel, dim3(mb), dim3(kBT), 0, s, qs, N, L, w, words);
    hipLaunchKernelGGL(ws2_walk_kernel, dim3(1), dim3(1), 0, s, w);
  }
  return hipGetLastError();
}

// The quantised 2-D coordinates sorted once per solve as keys q_y 2^32 + q_x
// (the order the sorted probe needs); keys is scratch of N entries.
__global__ void pair_keys_kernel(const uint32_t* __restrict__ q, int64_t N,
                                 uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (i < N) keys[i] = ((uint64_t)q[2 * i + 1] << 32) | (uint64_t)q[2 * i];
}

hipError_t launch_sort_2d(hipStream_t s, const uint32_t* q, int64_t N, uint64_t* keys,
                          uint64_t* q2_sorted, void* tmp, size_t tmp_bytes) {
  hipLaunchKernelGGL(pair_keys_kernel, dim3((unsigned)((N + kBT - 1) / kBT)), dim3(kBT), 0, s, q,
                     N, keys);
  return radix_sort_u64(s, keys, q2_sorted, nullptr, nullptr, N, 64, tmp, tmp_bytes);
}

// counts[0] = the distinct points of the sorted pairs, g(1).
hipError_t launch_count_sorted_2d(hipStream_t s, const uint64_t* q2_sorted, int64_t N,
                                  int64_t* counts) {
  const int nb = red_blocks(N);
  hipLaunchKernelGGL(count_runs_keys_kernel<uint64_t>, dim3(nb), dim3(kBT), 0, s, q2_sorted, N,
                     counts);
  hipLaunchKernelGGL(sum_counts_kernel, dim3(1), dim3(kBT), 0, s, nb, counts);
  return hipGetLastError();
}

hipError_t launch_count_2d(hipStream_t s, const uint32_t* q, int64_t N, uint64_t m,
                           uint64_t* keys, uint64_t* keys_sorted, void* tmp, size_t tmp_bytes,
                           int64_t* counts) {
  if (count_2d_uses_bitmap(N, m)) {
    const uint64_t ncx = 4294967295ull / m + 1ull;
    const int64_t nw = (int64_t)((grid_cells_2d(m) + 31) / 32);
    uint32_t* words = reinterpret_cast<uint32_t*>(keys);
    const unsigned zb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, (nw + kBT - 1) / kBT));
    hipLaunchKernelGGL(zero_words_kernel, dim3(zb), dim3(kBT), 0, s, words, nw);
    hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s,
                       reinterpret_cast<unsigned long long*>(counts), 1);
    const unsigned mb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (N + kBT - 1) / kBT));
    hipLaunchKernelGGL(mark_cells_kernel, dim3(mb), dim3(kBT), 0, s, q, N, m, magic_of(m), ncx,
                       nw, words);
    hipLaunchKernelGGL(popcount_words_kernel, dim3(zb), dim3(kBT), 0, s, (const uint32_t*)words,
                       nw, reinterpret_cast<unsigned long long*>(counts));
    return hipGetLastError();
  }
  const unsigned bits = key_bits(2, m);
  const int nb = red_blocks(N);
  hipError_t e;
  if (bits <= 32) {
    // ids of this width fit in 32 bits: half the bytes through the sort
    uint32_t* k32 = reinterpret_cast<uint32_t*>(keys);
    uint32_t* s32 = reinterpret_cast<uint32_t*>(keys_sorted);
    hipLaunchKernelGGL(cells32_kernel, dim3((unsigned)((N + kBT - 1) / kBT)), dim3(kBT), 0, s, q,
                       N, m, k32);
    e = radix_sort_u32(s, k32, s32, nullptr, nullptr, N, (int)bits, tmp, tmp_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(count_runs_keys_kernel<uint32_t>, dim3(nb), dim3(kBT), 0, s,
                       (const uint32_t*)s32, N, counts);
  } else {
    hipLaunchKernelGGL(cells_kernel, dim3((unsigned)((N + kBT - 1) / kBT)), dim3(kBT), 0, s, q, N,
                       2, m, keys);
    e = radix_sort_u64(s, keys, keys_sorted, nullptr, nullptr, N, (int)bits, tmp, tmp_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(count_runs_keys_kernel<uint64_t>, dim3(nb), dim3(kBT), 0, s,
                       (const uint64_t*)keys_sorted, N, counts);
  }
  hipLaunchKernelGGL(sum_counts_kernel, dim3(1), dim3(kBT), 0, s, nb, counts);
  return hipGetLastError();
}

// ---- histogram ----------------------------------------------------------------
__global__ void keys_from_sorted_1d_kernel(const uint32_t* __restrict__ qs, int64_t N, uint64_t m,
                                           uint64_t* __restrict__ ks) {
  const int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (i < N) ks[i] = (uint64_t)qs[i] / m;
}

__global__ void copy_u32_kernel(const uint32_t* __restrict__ a, int64_t N, uint32_t* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (i < N) b[i] = a[i];
}

__global__ void run_flags_kernel(const uint64_t* __restrict__ ks, int64_t N,
                                 int32_t* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (i < N) flags[i] = (i == 0) ? 1 : (ks[i] != ks[i - 1]);
}

// bin_of_pos holds the inclusive scan of the run flags on entry.
__global__ void run_starts_kernel(const uint64_t* __restrict__ ks, int64_t N,
                                  int32_t* __restrict__ bin_of_pos, int64_t* __restrict__ start,
                                  uint64_t* __restrict__ cells, int64_t* __restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (i >= N) return;
  const int32_t b = bin_of_pos[i] - 1;
  const bool first = (i == 0) || (ks[i] != ks[i - 1]);
  if (first) {
    start[b] = i;
    cells[b] = ks[i];
  }
  if (i == N - 1) {
    start[b + 1] = N;
    counts[0] = (int64_t)b + 1;
  }
  bin_of_pos[i] = b;
}

hipError_t launch_histogram(hipStream_t s, const uint32_t* q, int64_t N, int d, uint64_t m,
                            const uint32_t* q1_sorted, const uint32_t* perm1, uint32_t* iota,
                            uint64_t* keys, uint64_t* keys_sorted, uint32_t* perm,
                            int32_t* bin_of_pos, int64_t* start, uint64_t* cells, void* tmp,
                            size_t tmp_bytes, int64_t* counts) {
  const unsigned nb = (unsigned)((N + kBT - 1) / kBT);
  hipError_t e;
  if (d == 1) {
    hipLaunchKernelGGL(keys_from_sorted_1d_kernel, dim3(nb), dim3(kBT), 0, s, q1_sorted, N, m,
                       keys_sorted);
    hipLaunchKernelGGL(copy_u32_kernel, dim3(nb), dim3(kBT), 0, s, perm1, N, perm);
  } else {
    hipLaunchKernelGGL(cells_kernel, dim3(nb), dim3(kBT), 0, s, q, N, 2, m, keys);
    hipLaunchKernelGGL(iota_kernel, dim3(nb), dim3(kBT), 0, s, iota, N);
    e = radix_sort_u64(s, keys, keys_sorted, iota, perm, N, (int)key_bits(2, m), tmp, tmp_bytes);
    if (e != hipSuccess) return e;
  }
  // run flags -> inclusive scan -> bin index per sorted position
  int32_t* flags = reinterpret_cast<int32_t*>(keys);  // keys no longer needed
  hipLaunchKernelGGL(run_flags_kernel, dim3(nb), dim3(kBT), 0, s, keys_sorted, N, flags);
  e = scan_inclusive_i32(s, flags, bin_of_pos, N, tmp, tmp_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(run_starts_kernel, dim3(nb), dim3(kBT), 0, s, keys_sorted, N, bin_of_pos,
                     start, cells, counts);
  return hipGetLastError();
}

// ---- representatives ------------------------------------------------------------
// CENTRE (model): ubar_kp = u_k(centre of bin p), centre_j = lo_j + (c_j + 1/2) m / scale_j.
// MEAN (no model): ubar_kp = mean of u_kn over the bin's samples (sorted order,
// which is ascending sample index within a bin because the sort is stable).
__global__ void __launch_bounds__(kBT)
    represent_kernel(int K, int64_t N, int d, int model, const double* __restrict__ coef,
                     const double* __restrict__ lo, const double* __restrict__ scale, uint64_t m,
                     int64_t P, const uint64_t* __restrict__ cells,
                     const int64_t* __restrict__ start, const uint32_t* __restrict__ perm,
                     const double* __restrict__ u, double* __restrict__ ubar,
                     double* __restrict__ h) {
  const int64_t e = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (e >= (int64_t)K * P) return;
  const int k = (int)(e / P);
  const int64_t p = e % P;
  const int64_t s0 = start[p], s1 = start[p + 1];
  if (k == 0) h[p] = (double)(s1 - s0);
  double v;
  if (model == BUMBAR_MODEL_NONE) {
    double acc = 0.0;
    for (int64_t i = s0; i < s1; ++i) acc += u[(int64_t)k * N + perm[i]];
    v = acc / (double)(s1 - s0);
  } else {
    double x[2];
    uint64_t cc[2];
    if (d == 1) {
      cc[0] = cells[p];
    } else {
      const uint64_t stride = 4294967295ull / m + 1ull;
      cc[0] = cells[p] % stride;
      cc[1] = cells[p] / stride;
    }
    for (int j = 0; j < d; ++j)
      x[j] = scale[j] > 0.0 ? lo[j] + ((double)cc[j] + 0.5) * (double)m / scale[j] : lo[j];
    const double* ck = coef + (int64_t)k * (1 + 2 * d);
    v = ck[0];
    for (int j = 0; j < d; ++j) {
      if (model == BUMBAR_MODEL_LINEAR) {
        v += ck[1 + j] * x[j];
      } else {
        const double dx = x[j] - ck[2 + 2 * j];
        v += 0.5 * ck[1 + 2 * j] * dx * dx;
      }
    }
  }
  ubar[(int64_t)k * P + p] = v;
}

hipError_t launch_represent(hipStream_t s, int K, int64_t N, int d, int model, const double* coef,
                            const double* lo, const double* scale, uint64_t m, int64_t P,
                            const uint64_t* cells, const int64_t* start, const uint32_t* perm,
                            const double* u, double* ubar, double* h) {
  const int64_t tot = (int64_t)K * P;
  hipLaunchKernelGGL(represent_kernel, dim3((unsigned)((tot + kBT - 1) / kBT)), dim3(kBT), 0, s, K,
                     N, d, model, coef, lo, scale, m, P, cells, start, perm, u, ubar, h);
  return hipGetLastError();
}

// The same bin-centre representatives in the sample-major layout of the
// 256 < K <= 1024 sweeps: row p holds the Kp values model_k(centre_p) (+inf
// past K), from the centres of centres_kernel and the arithmetic of
// represent_kernel, so the values are those of the state-major form.
__global__ void __launch_bounds__(kBT)
    represent_smaj_kernel(int K, int Kp, int d, int model, const double* __restrict__ coef,
                          int64_t P, const double* __restrict__ cen, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (e >= (int64_t)Kp * P) return;
  const int64_t p = e / Kp;
  const int k = (int)(e % Kp);
  if (k >= K) {
    out[e] = INFINITY;
    return;
  }
  const double* ck = coef + (int64_t)k * (1 + 2 * d);
  double v = ck[0];
  for (int j = 0; j < d; ++j) {
    const double x = cen[p * d + j];
    if (model == BUMBAR_MODEL_LINEAR) {
      v += ck[1 + j] * x;
    } else {
      const double dx = x - ck[2 + 2 * j];
      v += 0.5 * ck[1 + 2 * j] * dx * dx;
    }
  }
  out[e] = v;
}

hipError_t launch_represent_smaj(hipStream_t s, int K, int Kp, int d, int model,
                                 const double* coef, int64_t P, const double* cen, double* out) {
  const int64_t tot = (int64_t)Kp * P;
  hipLaunchKernelGGL(represent_smaj_kernel, dim3((unsigned)((tot + kBT - 1) / kBT)), dim3(kBT), 0,
                     s, K, Kp, d, model, coef, P, cen, out);
  return hipGetLastError();
}

// Bin centres (P x d) and multiplicities of the current histogram: the
// coordinates at which the bias model gives the bin representative (the
// same centre as in represent_kernel), for sweeps that evaluate the model
// inside the kernel instead of storing K x P representatives.
__global__ void centres_kernel(int d, const double* __restrict__ lo,
                               const double* __restrict__ scale, uint64_t m, int64_t P,
                               const uint64_t* __restrict__ cells,
                               const int64_t* __restrict__ start, double* __restrict__ cen,
                               double* __restrict__ h) {
  const int64_t p = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (p >= P) return;
  h[p] = (double)(start[p + 1] - start[p]);
  uint64_t cc[2];
  if (d == 1) {
    cc[0] = cells[p];
    cc[1] = 0;
  } else {
    const uint64_t stride = 4294967295ull / m + 1ull;
    cc[0] = cells[p] % stride;
    cc[1] = cells[p] / stride;
  }
  for (int j = 0; j < d; ++j)
    cen[p * d + j] = scale[j] > 0.0 ? lo[j] + ((double)cc[j] + 0.5) * (double)m / scale[j] : lo[j];
}

hipError_t launch_centres(hipStream_t s, int d, const double* lo, const double* scale, uint64_t m,
                          int64_t P, const uint64_t* cells, const int64_t* start, double* cen,
                          double* h) {
  hipLaunchKernelGGL(centres_kernel, dim3((unsigned)((P + kBT - 1) / kBT)), dim3(kBT), 0, s, d, lo,
                     scale, m, P, cells, start, cen, h);
  return hipGetLastError();
}

__global__ void sample_bin_kernel(int64_t N, const uint32_t* __restrict__ perm,
                                  const int32_t* __restrict__ bin_of_pos,
                                  int32_t* __restrict__ sample_bin) {
  const int64_t i = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (i < N) sample_bin[perm[i]] = bin_of_pos[i];
}

hipError_t launch_sample_bin(hipStream_t s, int64_t N, const uint32_t* perm,
                             const int32_t* bin_of_pos, int32_t* sample_bin) {
  hipLaunchKernelGGL(sample_bin_kernel, dim3((unsigned)((N + kBT - 1) / kBT)), dim3(kBT), 0, s, N,
                     perm, bin_of_pos, sample_bin);
  return hipGetLastError();
}

__global__ void counts_from_start_kernel(int64_t P, const int64_t* __restrict__ start,
                                         int64_t* __restrict__ H) {
  const int64_t p = (int64_t)blockIdx.x * kBT + threadIdx.x;
  if (p < P) H[p] = start[p + 1] - start[p];
}

hipError_t launch_counts_from_start(hipStream_t s, int64_t P, const int64_t* start, int64_t* H) {
  hipLaunchKernelGGL(counts_from_start_kernel, dim3((unsigned)((P + kBT - 1) / kBT)), dim3(kBT), 0,
                     s, P, start, H);
  return hipGetLastError();
}

}  // namespace bumbar
