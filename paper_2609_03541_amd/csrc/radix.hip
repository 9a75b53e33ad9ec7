// Integer sorting and scanning for the binning (Section 2, text after
// Eq. (1): the bins are the distinct cells of the quantised coordinates and
// H_p their counts), written for gfx950.
//
// Stable LSD radix sort of 32- or 64-bit keys, optionally carrying a 32-bit
// value, over the low `bits` bits, 8 bits per pass. A pass over tiles of
// kTile = 16 x 256 keys:
//   1. histogram: each workgroup counts the digits of its tile in a 256-bin
//      LDS histogram (integer atomics) and writes it digit-major,
//      hist[d * nb + b];
//   2. exclusive scan of hist (digit-major order): the first output position
//      of digit d for tile b;
//   3. scatter: each workgroup walks its tile in 16 rounds of 256 keys (key
//      i = b kTile + 256 j + t in round j); a key's rank among the keys of its
//      digit before it is the digit's running count, plus the counts of the
//      earlier waves of the round (LDS), plus the lanes of its own wave with
//      the same digit below it (eight ballots over the digit's bits, then a
//      popcount). Equal digits keep their input order, so every pass, and the
//      sort, is stable.
// Scan: three launches (per-block sums, a one-workgroup scan of the block
// sums, per-block scans plus their offsets); integer, so exact.
//
// Small inputs (at most kSmallTiles tiles, or kSmallScan scan chunks) run the
// same steps in one workgroup and one launch: every pass keeps all tile
// histograms in LDS, and the workgroup barrier between passes orders each
// pass's scattered stores before the next pass reads them. A sort of 8000
// keys is then one launch instead of five per pass.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "bumbar_impl.h"

namespace bumbar {

namespace {

constexpr int kRT = 256;             // threads of a radix workgroup
constexpr int kRounds = 16;          // keys per thread per tile
constexpr int kTile = kRT * kRounds; // keys per tile
constexpr int kST = 256;             // threads of a scan workgroup
constexpr int kSItems = 8;           // items per scan thread
constexpr int kSChunk = kST * kSItems;

constexpr int kSmallTiles = 16;      // one-workgroup sorts: up to 16 tiles (65536 keys)
constexpr int kSmallScan = 4;        // one-workgroup scans: up to 4 chunks (8192 items)

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

__host__ __device__ int64_t radix_tiles(int64_t N) { return (N + kTile - 1) / kTile; }
int64_t scan_blocks(int64_t n) { return (n + kSChunk - 1) / kSChunk; }

template <typename K>
__device__ __forceinline__ unsigned digit_of(K k, int shift) {
  return (unsigned)((k >> shift) & (K)0xff);
}

template <typename K>
__global__ void __launch_bounds__(kRT)
    radix_hist_kernel(const K* __restrict__ src, int64_t N, int shift, int64_t nb,
                      uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const int t = threadIdx.x;
  h[t] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll 4
  for (int j = 0; j < kRounds; ++j) {
    const int64_t i = base + (int64_t)j * kRT + t;
    if (i < N) atomicAdd(&h[digit_of(src[i], shift)], 1u);
  }
  __syncthreads();
  hist[(int64_t)t * nb + blockIdx.x] = h[t];
}

template <typename K, bool VALS>
__global__ void __launch_bounds__(kRT)
    radix_scatter_kernel(const K* __restrict__ src, const uint32_t* __restrict__ vsrc, int64_t N,
                         int shift, int64_t nb, const uint32_t* __restrict__ offs,
                         K* __restrict__ dst, uint32_t* __restrict__ vdst) {
  __shared__ uint32_t running[256];
  __shared__ uint32_t cnt[kRT / 64][256];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  running[t] = offs[(int64_t)t * nb + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kRT / 64; ++w) cnt[w][t] = 0u;
  __syncthreads();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kTile;
  // the thread's keys (and values) of the tile, loaded together
  K kr[kRounds];
  uint32_t vr[kRounds];
#pragma unroll
  for (int j = 0; j < kRounds; ++j) {
    const int64_t i = base + (int64_t)j * kRT + t;
    kr[j] = i < N ? src[i] : (K)0;
    if constexpr (VALS) vr[j] = i < N ? vsrc[i] : 0u;
  }
#pragma unroll
  for (int j = 0; j < kRounds; ++j) {
    const int64_t i = base + (int64_t)j * kRT + t;
    const bool valid = i < N;
    const K key = kr[j];
    const unsigned d = digit_of(key, shift);
    // lanes of this wave holding a valid key with the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t b = __ballot(valid && ((d >> bit) & 1u));
      peers &= ((d >> bit) & 1u) ? b : ~b;
    }
    const unsigned rank = (unsigned)__popcll(peers & below);
    if (valid && rank == 0u) cnt[wave][d] = (unsigned)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = running[d] + rank;
      for (int w = 0; w < wave; ++w) pos += cnt[w][d];
      dst[pos] = key;
      if constexpr (VALS) vdst[pos] = vr[j];
    }
    __syncthreads();
    uint32_t add = 0u;
#pragma unroll
    for (int w = 0; w < kRT / 64; ++w) {
      add += cnt[w][t];
      cnt[w][t] = 0u;
    }
    running[t] += add;
    __syncthreads();
  }
}

// All passes of a sort of at most kSmallTiles tiles in one workgroup: the
// digit histograms of every tile in LDS, their digit-major exclusive scan,
// and the scatter of each tile in turn, exactly as the three kernels above
// compute them. Pass p reads what pass p - 1 wrote; the barrier at the end of
// a pass orders those stores (all within this workgroup) before the loads.
template <typename K, bool VALS>
__global__ void __launch_bounds__(kRT)
    radix_small_kernel(const K* keys_in, const uint32_t* vals_in, K* keys_out,
                       uint32_t* vals_out, K* kalt, uint32_t* valt, int64_t N, int passes) {
  __shared__ uint32_t h[kSmallTiles][256];
  __shared__ uint32_t dsum[256];
  __shared__ uint32_t running[256];
  __shared__ uint32_t cnt[kRT / 64][256];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int nb = (int)radix_tiles(N);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const K* ks = keys_in;
  const uint32_t* vs = vals_in;
  for (int p = 0; p < passes; ++p) {
    // the last pass writes keys_out
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    K* kd = to_out ? keys_out : kalt;
    uint32_t* vd = to_out ? vals_out : valt;
    const int shift = 8 * p;
    for (int b = 0; b < nb; ++b) h[b][t] = 0u;
    __syncthreads();
#pragma unroll 8
    for (int64_t i = t; i < N; i += kRT) atomicAdd(&h[i / kTile][digit_of(ks[i], shift)], 1u);
    __syncthreads();
    // first output position of digit t in tile b: the keys of smaller digits,
    // then those of digit t in earlier tiles
    uint32_t tot = 0u;
    for (int b = 0; b < nb; ++b) tot += h[b][t];
    dsum[t] = tot;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t a = t >= off ? dsum[t - off] : 0u;
      __syncthreads();
      dsum[t] += a;
      __syncthreads();
    }
    uint32_t run = dsum[t] - tot;
    for (int b = 0; b < nb; ++b) {
      const uint32_t c = h[b][t];
      h[b][t] = run;
      run += c;
    }
    for (int b = 0; b < nb; ++b) {
      running[t] = h[b][t];
#pragma unroll
      for (int w = 0; w < kRT / 64; ++w) cnt[w][t] = 0u;
      // the tile's keys (and values) of this thread, loaded together: the
      // rounds below then wait on no memory
      const int64_t base = (int64_t)b * kTile;
      K kr[kRounds];
      uint32_t vr[kRounds];
#pragma unroll
      for (int j = 0; j < kRounds; ++j) {
        const int64_t i = base + (int64_t)j * kRT + t;
        kr[j] = i < N ? ks[i] : (K)0;
        if constexpr (VALS) vr[j] = i < N ? vs[i] : 0u;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kRounds; ++j) {
        const int64_t i = base + (int64_t)j * kRT + t;
        const bool valid = i < N;
        const K key = kr[j];
        const unsigned d = digit_of(key, shift);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
          const uint64_t bb = __ballot(valid && ((d >> bit) & 1u));
          peers &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const unsigned rank = (unsigned)__popcll(peers & below);
        if (valid && rank == 0u) cnt[wave][d] = (unsigned)__popcll(peers);
        __syncthreads();
        if (valid) {
          uint32_t pos = running[d] + rank;
          for (int w = 0; w < wave; ++w) pos += cnt[w][d];
          kd[pos] = key;
          if constexpr (VALS) vd[pos] = vr[j];
        }
        __syncthreads();
        uint32_t add = 0u;
#pragma unroll
        for (int w = 0; w < kRT / 64; ++w) {
          add += cnt[w][t];
          cnt[w][t] = 0u;
        }
        running[t] += add;
        __syncthreads();
      }
    }
    __syncthreads();
    ks = kd;
    vs = vd;
  }
}

// ---- scan ----------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* sh, T* total) {
  // inclusive scan across the workgroup through LDS (Hillis-Steele), then
  // shifted to exclusive
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kST; off <<= 1) {
    const T a = t >= off ? sh[t - off] : (T)0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const T inc = sh[t];
  *total = sh[kST - 1];
  __syncthreads();
  return inc - v;
}

template <typename T>
__global__ void __launch_bounds__(kST)
    scan_sums_kernel(const T* in, int64_t n, T* __restrict__ sums) {
  __shared__ T sh[kST];
  const int64_t base = (int64_t)blockIdx.x * kSChunk + (int64_t)threadIdx.x * kSItems;
  T v = 0;
#pragma unroll
  for (int q = 0; q < kSItems; ++q)
    if (base + q < n) v += in[base + q];
  T tot;
  (void)block_exclusive_scan<T>(v, sh, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// one workgroup: exclusive scan of the m block sums in place
template <typename T>
__global__ void __launch_bounds__(kST) scan_top_kernel(T* __restrict__ sums, int64_t m) {
  __shared__ T sh[kST];
  const int64_t per = (m + kST - 1) / kST;
  const int64_t b0 = (int64_t)threadIdx.x * per;
  T v = 0;
  for (int64_t q = 0; q < per; ++q)
    if (b0 + q < m) v += sums[b0 + q];
  T tot;
  T run = block_exclusive_scan<T>(v, sh, &tot);
  for (int64_t q = 0; q < per; ++q)
    if (b0 + q < m) {
      const T x = sums[b0 + q];
      sums[b0 + q] = run;
      run += x;
    }
}

template <typename T, bool INCLUSIVE>
__global__ void __launch_bounds__(kST)
    scan_apply_kernel(const T* in, int64_t n, const T* __restrict__ sums, T* out) {
  // in and out may be the same array (the digit counts are scanned in place):
  // each thread reads its items before the workgroup scan and writes them after
  __shared__ T sh[kST];
  const int64_t base = (int64_t)blockIdx.x * kSChunk + (int64_t)threadIdx.x * kSItems;
  T x[kSItems];
  T v = 0;
#pragma unroll
  for (int q = 0; q < kSItems; ++q) {
    x[q] = base + q < n ? in[base + q] : (T)0;
    v += x[q];
  }
  T tot;
  T run = block_exclusive_scan<T>(v, sh, &tot) + sums[blockIdx.x];
#pragma unroll
  for (int q = 0; q < kSItems; ++q) {
    if (INCLUSIVE) run += x[q];
    if (base + q < n) out[base + q] = run;
    if (!INCLUSIVE) run += x[q];
  }
}

// One workgroup over at most kSmallScan chunks, each scanned as by
// scan_apply_kernel with the running total of the chunks before it. In place
// as well: every item is read before the first one is written.
template <typename T, bool INCLUSIVE>
__global__ void __launch_bounds__(kST) scan_small_kernel(const T* in, int64_t n, T* out) {
  __shared__ T sh[kST];
  // every item of this thread, all chunks, loaded before the first scan
  T x[kSmallScan][kSItems];
#pragma unroll
  for (int c = 0; c < kSmallScan; ++c) {
    const int64_t base = (int64_t)c * kSChunk + (int64_t)threadIdx.x * kSItems;
#pragma unroll
    for (int q = 0; q < kSItems; ++q) x[c][q] = base + q < n ? in[base + q] : (T)0;
  }
  T carry = 0;
#pragma unroll
  for (int c = 0; c < kSmallScan; ++c) {
    if ((int64_t)c * kSChunk >= n) break;  // uniform
    const int64_t base = (int64_t)c * kSChunk + (int64_t)threadIdx.x * kSItems;
    T v = 0;
#pragma unroll
    for (int q = 0; q < kSItems; ++q) v += x[c][q];
    T tot;
    T run = block_exclusive_scan<T>(v, sh, &tot) + carry;
#pragma unroll
    for (int q = 0; q < kSItems; ++q) {
      if (INCLUSIVE) run += x[c][q];
      if (base + q < n) out[base + q] = run;
      if (!INCLUSIVE) run += x[c][q];
    }
    carry += tot;
  }
}

template <typename T, bool INCLUSIVE>
hipError_t scan_t(hipStream_t s, const T* in, T* out, int64_t n, T* sums) {
  if (n <= 0) return hipSuccess;
  const int64_t nbk = scan_blocks(n);
  if (nbk <= kSmallScan) {
    hipLaunchKernelGGL((scan_small_kernel<T, INCLUSIVE>), dim3(1), dim3(kST), 0, s, in, n, out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(scan_sums_kernel<T>, dim3((unsigned)nbk), dim3(kST), 0, s, in, n, sums);
  hipLaunchKernelGGL(scan_top_kernel<T>, dim3(1), dim3(kST), 0, s, sums, nbk);
  hipLaunchKernelGGL((scan_apply_kernel<T, INCLUSIVE>), dim3((unsigned)nbk), dim3(kST), 0, s, in,
                     n, (const T*)sums, out);
  return hipGetLastError();
}

template <typename K>
hipError_t radix_sort_t(hipStream_t s, const K* keys_in, K* keys_out, const uint32_t* vals_in,
                        uint32_t* vals_out, int64_t N, int bits, void* tmp, size_t tmp_bytes) {
  if (N <= 0) return hipSuccess;
  if (N > 0xffffffffll || bits < 0 || bits > (int)(8 * sizeof(K)) ||
      tmp_bytes < radix_temp_bytes(N) || (vals_in != nullptr) != (vals_out != nullptr))
    return hipErrorInvalidValue;
  const int64_t nb = radix_tiles(N);
  char* w = static_cast<char*>(tmp);
  K* kalt = reinterpret_cast<K*>(w);
  w += al256(sizeof(uint64_t) * (size_t)N);
  uint32_t* valt = reinterpret_cast<uint32_t*>(w);
  w += al256(sizeof(uint32_t) * (size_t)N);
  uint32_t* hist = reinterpret_cast<uint32_t*>(w);
  w += al256(sizeof(uint32_t) * 256 * (size_t)nb);
  uint32_t* sums = reinterpret_cast<uint32_t*>(w);
  const int passes = (bits + 7) / 8;
  const bool vals = vals_in != nullptr;
  if (passes == 0) {
    hipError_t e = hipMemcpyAsync(keys_out, keys_in, sizeof(K) * (size_t)N,
                                  hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && vals)
      e = hipMemcpyAsync(vals_out, vals_in, sizeof(uint32_t) * (size_t)N,
                         hipMemcpyDeviceToDevice, s);
    return e;
  }
  if (nb <= kSmallTiles) {
    if (vals)
      hipLaunchKernelGGL((radix_small_kernel<K, true>), dim3(1), dim3(kRT), 0, s, keys_in, vals_in,
                         keys_out, vals_out, kalt, valt, N, passes);
    else
      hipLaunchKernelGGL((radix_small_kernel<K, false>), dim3(1), dim3(kRT), 0, s, keys_in,
                         (const uint32_t*)nullptr, keys_out, (uint32_t*)nullptr, kalt,
                         (uint32_t*)nullptr, N, passes);
    return hipGetLastError();
  }
  // the last pass writes keys_out: an odd count starts there
  const K* ks = keys_in;
  const uint32_t* vs = vals_in;
  for (int p = 0; p < passes; ++p) {
    const bool to_out = ((passes - 1 - p) % 2) == 0;
    K* kd = to_out ? keys_out : kalt;
    uint32_t* vd = to_out ? vals_out : valt;
    const int shift = 8 * p;
    hipLaunchKernelGGL(radix_hist_kernel<K>, dim3((unsigned)nb), dim3(kRT), 0, s, ks, N, shift,
                       nb, hist);
    hipError_t e = scan_t<uint32_t, false>(s, hist, hist, 256 * nb, sums);
    if (e != hipSuccess) return e;
    if (vals)
      hipLaunchKernelGGL((radix_scatter_kernel<K, true>), dim3((unsigned)nb), dim3(kRT), 0, s, ks,
                         vs, N, shift, nb, (const uint32_t*)hist, kd, vd);
    else
      hipLaunchKernelGGL((radix_scatter_kernel<K, false>), dim3((unsigned)nb), dim3(kRT), 0, s,
                         ks, (const uint32_t*)nullptr, N, shift, nb, (const uint32_t*)hist, kd,
                         (uint32_t*)nullptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ks = kd;
    vs = vd;
  }
  return hipSuccess;
}

}  // namespace

size_t radix_temp_bytes(int64_t N) {
  const int64_t nb = radix_tiles(N);
  return al256(sizeof(uint64_t) * (size_t)N) + al256(sizeof(uint32_t) * (size_t)N) +
         al256(sizeof(uint32_t) * 256 * (size_t)nb) +
         al256(sizeof(uint32_t) * (size_t)scan_blocks(256 * nb)) + 256;
}

size_t scan_temp_bytes(int64_t N) { return al256(sizeof(int64_t) * (size_t)scan_blocks(N)) + 256; }

hipError_t radix_sort_u32(hipStream_t s, const uint32_t* keys_in, uint32_t* keys_out,
                          const uint32_t* vals_in, uint32_t* vals_out, int64_t N, int bits,
                          void* tmp, size_t tmp_bytes) {
  return radix_sort_t<uint32_t>(s, keys_in, keys_out, vals_in, vals_out, N, bits, tmp, tmp_bytes);
}

hipError_t radix_sort_u64(hipStream_t s, const uint64_t* keys_in, uint64_t* keys_out,
                          const uint32_t* vals_in, uint32_t* vals_out, int64_t N, int bits,
                          void* tmp, size_t tmp_bytes) {
  return radix_sort_t<uint64_t>(s, keys_in, keys_out, vals_in, vals_out, N, bits, tmp, tmp_bytes);
}

hipError_t scan_inclusive_i32(hipStream_t s, const int32_t* in, int32_t* out, int64_t N,
                              void* tmp, size_t tmp_bytes) {
  if (tmp_bytes < scan_temp_bytes(N)) return hipErrorInvalidValue;
  return scan_t<int32_t, true>(s, in, out, N, static_cast<int32_t*>(tmp));
}

}  // namespace bumbar
