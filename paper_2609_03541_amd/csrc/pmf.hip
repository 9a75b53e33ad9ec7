// Free-energy surface on a regular grid of the sampled coordinates (Section 3,
// Eqs. (5)-(6): the per-sample probabilities p_n at a target state; the
// surfaces of Fig. 1 are -ln of their sums over coordinate bins).
//
// F_b = -ln sum_{n in bin b} p_n. Sample n falls in bin b = sum_j b_j s_j
// (row-major, the first coordinate slowest) with
//   b_j = floor((xi_nj - lo_j) * nb_j / (hi_j - lo_j)),
// evaluated in FP64 in exactly that order, and is left out unless
// 0 <= b_j < nb_j for every j. The bin ids are radix-sorted together with the
// sample index (a stable sort keeps equal ids in index order), so each bin is
// a run of its samples in ascending n. A run is summed in segments of at most
// kSeg sorted positions (cut at multiples of kSeg), each added in order by
// one thread, and the thread at the run's start then adds its segments in
// order. The order of additions depends only on the data, not on the launch,
// and no thread walks more than kSeg samples plus one sum per segment.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "bumbar_impl.h"
#include "solver_internal.h"

namespace bumbar {

constexpr int kPT = 256;

// key[n] = bin of sample n, or nbins (one past the last bin) when it is
// outside the grid; val[n] = n.
__global__ void __launch_bounds__(kPT)
    pmf_bin_kernel(const double* __restrict__ xi, int64_t N, int d, double lo0, double hi0,
                   int nb0, double lo1, double hi1, int nb1, uint32_t nbins,
                   uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
  const int64_t n = (int64_t)blockIdx.x * kPT + threadIdx.x;
  if (n >= N) return;
  uint32_t b = nbins;
  const double b0 = floor((xi[n * d] - lo0) * (double)nb0 / (hi0 - lo0));
  if (b0 >= 0.0 && b0 < (double)nb0) {
    if (d == 1) {
      b = (uint32_t)b0;
    } else {
      const double b1 = floor((xi[n * d + 1] - lo1) * (double)nb1 / (hi1 - lo1));
      if (b1 >= 0.0 && b1 < (double)nb1) b = (uint32_t)b0 * (uint32_t)nb1 + (uint32_t)b1;
    }
  }
  key[n] = b;
  val[n] = (uint32_t)n;
}

__global__ void __launch_bounds__(kPT) pmf_fill_kernel(double* __restrict__ F, int64_t nbins) {
  const int64_t b = (int64_t)blockIdx.x * kPT + threadIdx.x;
  if (b < nbins) F[b] = INFINITY;
}

constexpr int64_t kSeg = 1024;  // sorted positions per segment

// The thread at the start of each segment (the start of a run, or a multiple
// of kSeg inside one) adds the segment's probabilities in order.
__global__ void __launch_bounds__(kPT)
    pmf_segments_kernel(const uint32_t* __restrict__ ks, const uint32_t* __restrict__ vs,
                        int64_t N, uint32_t nbins, const double* __restrict__ p,
                        double* __restrict__ seg) {
  const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
  if (i >= N) return;
  const uint32_t k = ks[i];
  if (k >= nbins || (i % kSeg != 0 && ks[i - 1] == k)) return;
  const int64_t end = (i / kSeg + 1) * kSeg < N ? (i / kSeg + 1) * kSeg : N;
  double s = 0.0;
  for (int64_t j = i; j < end && ks[j] == k; ++j) s += p[vs[j]];
  seg[i] = s;
}

// The thread at the start of each run adds the run's segment sums in order.
__global__ void __launch_bounds__(kPT)
    pmf_runs_kernel(const uint32_t* __restrict__ ks, int64_t N, uint32_t nbins,
                    const double* __restrict__ seg, double* __restrict__ F) {
  const int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
  if (i >= N) return;
  const uint32_t k = ks[i];
  if (k >= nbins || (i > 0 && ks[i - 1] == k)) return;
  double s = seg[i];
  for (int64_t c = (i / kSeg + 1) * kSeg; c < N && ks[c] == k; c += kSeg) s += seg[c];
  F[k] = -log(s);
}

static unsigned pmf_key_bits(uint32_t nbins) {
  unsigned b = 1;
  while (b < 32 && (uint64_t)nbins >> b) ++b;
  return b;
}

static size_t pmf_sort_bytes(int64_t N) { return radix_temp_bytes(N); }

static size_t pmf_align(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace bumbar

using namespace bumbar;

extern "C" {

int bumbar_query_workspace_pmf(const bumbar_ctx* ctx, int64_t N, size_t* bytes) {
  if (!ctx || !bytes || N <= 0 || N > 0xffffffffll) return BUMBAR_EINVAL;
  *bytes = 4 * pmf_align(sizeof(uint32_t) * (size_t)N) + pmf_align(sizeof(double) * (size_t)N) +
           pmf_align(pmf_sort_bytes(N)) + 256;
  return BUMBAR_OK;
}

int bumbar_pmf(bumbar_ctx* ctx, const double* xi, int64_t N, int d, const double* p,
               const double* lo, const double* hi, const int* nbins, void* workspace,
               size_t ws_bytes, double* F) {
  if (!ctx) return BUMBAR_EINVAL;
  ctx->err.clear();
  if (!xi || !p || !lo || !hi || !nbins || !workspace || !F || N <= 0 || N > 0xffffffffll ||
      (d != 1 && d != 2))
    return fail(ctx, BUMBAR_EINVAL, "bad argument");
  int64_t total = 1;
  for (int j = 0; j < d; ++j) {
    if (nbins[j] < 1 || !(hi[j] > lo[j]) || !std::isfinite(lo[j]) || !std::isfinite(hi[j]))
      return fail(ctx, BUMBAR_EINVAL, "grid dimension %d: need nbins >= 1 and finite lo < hi", j);
    total *= nbins[j];
  }
  if (total >= 0xffffffffll) return fail(ctx, BUMBAR_EINVAL, "too many bins");
  size_t need = 0;
  (void)bumbar_query_workspace_pmf(ctx, N, &need);
  if (ws_bytes < need) return fail(ctx, BUMBAR_ENOMEM, "workspace too small (%zu, need %zu)",
                                   ws_bytes, need);
  char* w = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(workspace) + 255) & ~uintptr_t(255));
  const size_t a = pmf_align(sizeof(uint32_t) * (size_t)N);
  uint32_t* key = reinterpret_cast<uint32_t*>(w);
  uint32_t* val = reinterpret_cast<uint32_t*>(w + a);
  uint32_t* ks = reinterpret_cast<uint32_t*>(w + 2 * a);
  uint32_t* vs = reinterpret_cast<uint32_t*>(w + 3 * a);
  double* seg = reinterpret_cast<double*>(w + 4 * a);
  void* tmp = w + 4 * a + pmf_align(sizeof(double) * (size_t)N);
  size_t tmp_bytes = pmf_sort_bytes(N);
  hipStream_t s = ctx->stream;
  const uint32_t nb = (uint32_t)total;
  const unsigned blocks = (unsigned)((N + kPT - 1) / kPT);
  hipLaunchKernelGGL(pmf_bin_kernel, dim3(blocks), dim3(kPT), 0, s, xi, N, d, lo[0], hi[0],
                     nbins[0], d == 2 ? lo[1] : 0.0, d == 2 ? hi[1] : 1.0, d == 2 ? nbins[1] : 1,
                     nb, key, val);
  hipLaunchKernelGGL(pmf_fill_kernel, dim3((unsigned)((total + kPT - 1) / kPT)), dim3(kPT), 0, s,
                     F, total);
  hipError_t e = radix_sort_u32(s, key, ks, val, vs, N, (int)pmf_key_bits(nb), tmp, tmp_bytes);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(pmf_segments_kernel, dim3(blocks), dim3(kPT), 0, s, ks, vs, N, nb, p, seg);
    hipLaunchKernelGGL(pmf_runs_kernel, dim3(blocks), dim3(kPT), 0, s, ks, N, nb, seg, F);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "pmf");
  return BUMBAR_OK;
}

}  // extern "C"
