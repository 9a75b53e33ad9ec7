// Hessian of the MBAR objective on FP64 matrix cores (gfx950 MFMA).
//
// F(f) = sum_n ln D_n - sum_k N_k f_k has gradient g_i = S_i - N_i and Hessian
//   H_ij = delta_ij S_i - sum_n P_in P_jn,   P_in = N_i W_ni = g_i exp(c_i - u_in - ln D_n)
// with c_i = ln N'_i + f_i (Section 2: derivative-based strategies; the Newton
// finisher on unbinned data). The contraction G = P P^T over the N samples is
// the only dense-matrix work of the method and runs on v_mfma_f64_16x16x4.
//
// Layout: the K x K output is cut into 64 x 64 blocks; only blocks with
// bi <= bj are computed (symmetry). A workgroup (4 waves) owns one block and
// one contiguous chunk of samples; per step of 16 samples it reads the two
// 64-row slabs of u (coalesced along n), forms P in registers (one exp per
// element), stages it in LDS, and each wave accumulates a 32 x 32 quarter of
// the block as 2 x 2 MFMA tiles. Partial blocks are summed over chunks in a
// fixed order by a second kernel, so the result is deterministic.
#include <cmath>
#include <type_traits>

#include "bumbar_impl.h"
#include "devmath.h"

namespace bumbar {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int HB = 64;   // output block edge
constexpr int HS = 16;   // samples per step
constexpr int HP = HS + 1;  // padded LDS row (doubles)

// Block index b in [0, nb*(nb+1)/2) -> (bi, bj) with bi <= bj, row-major over bi.
__device__ __forceinline__ void block_coords(int b, int nb, int& bi, int& bj) {
  int i = 0;
  int rem = b;
  while (rem >= nb - i) {
    rem -= nb - i;
    ++i;
  }
  bi = i;
  bj = i + rem;
}

// Sources of P_kn = g_k exp(c_k - u_kn - ln D_n) for one row k and one
// sample n: row(k, c) captures what is fixed along the row, col(n) what is
// fixed along the column, and p(row, n, col) the element.

// Stored FP64 or FP32 u: x = c_k - u_kn - ln D_n.
template <typename TI>
struct SrcMat {
  const TI* u;
  int64_t ld;
  struct Row {
    const TI* p;
    double c;
  };
  __device__ Row row(int k, double c) const { return {u + (int64_t)k * ld, c}; }
  __device__ double col(int64_t n, const double* logD) const { return logD[n]; }
  // p in two stages (the load, then the arithmetic), so that a kernel can
  // issue the next samples' loads before it consumes them
  using Raw = TI;
  __device__ Raw load(const Row& r, int64_t n) const { return r.p[n]; }
  __device__ double fin(const Row& r, Raw x, double lD) const {
    return exp_nonpos(r.c - (double)x - lD);
  }
  __device__ double p(const Row& r, int64_t n, double lD) const { return fin(r, load(r, n), lD); }
};

// FP64 u with the weight's exponential on the FP32 hardware exp2 (relative
// error about 1e-7): for the Newton Hessian, which only shapes the steps.
// The exponent c_k - u_kn - ln D_n is taken in FP64 and is <= 0.
struct SrcMatExp32 {
  const double* u;
  int64_t ld;
  struct Row {
    const double* p;
    double c;
  };
  __device__ Row row(int k, double c) const { return {u + (int64_t)k * ld, c}; }
  __device__ double col(int64_t n, const double* logD) const { return logD[n]; }
  using Raw = double;
  __device__ Raw load(const Row& r, int64_t n) const { return r.p[n]; }
  __device__ double fin(const Row& r, Raw x, double lD) const {
    return (double)__builtin_amdgcn_exp2f((float)(1.4426950408889634 * (r.c - x - lD)));
  }
  __device__ double p(const Row& r, int64_t n, double lD) const { return fin(r, load(r, n), lD); }
};

// Packed mixed-precision matrix r_kn = c0_k - u_kn - m0_n: x = d_k + r_kn -
// (ln D_n - m0_n) with d_k = c_k - c0_k passed as the row constant.
struct SrcPacked {
  const float* r;
  int64_t ld;
  const double* m0;
  struct Row {
    const float* p;
    double c;
  };
  __device__ Row row(int k, double c) const { return {r + (int64_t)k * ld, c}; }
  __device__ double col(int64_t n, const double* logD) const { return logD[n] - m0[n]; }
  __device__ double p(const Row& rw, int64_t n, double lD) const {
    return exp_nonpos(rw.c + (double)rw.p[n] - lD);
  }
};

// Energies from the bias model in FP64 (direct form), coordinates xi (N x D);
// c64 holds [E_col | E_st | H | X0] as built for the on-the-fly sweeps.
template <int D, int MODEL>
struct SrcModel64 {
  const double* xi;
  const double* c64;
  int K;
  struct Row {
    double e, h[D], x0[D];
  };
  __device__ Row row(int k, double) const {
    Row r;
    r.e = c64[K + k];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      r.h[j] = c64[2 * K + (int64_t)j * K + k];
      r.x0[j] = c64[2 * K + (int64_t)(D + j) * K + k];
    }
    return r;
  }
  __device__ double col(int64_t n, const double* logD) const { return logD[n]; }
  __device__ double p(const Row& r, int64_t n, double lD) const {
    double q = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const double x = xi[n * D + j];
      if (MODEL == BUMBAR_MODEL_HARMONIC) {
        const double dx = x - r.x0[j];
        q = __builtin_fma(r.h[j] * dx, dx, q);
      } else {
        q = __builtin_fma(r.h[j], x, q);
      }
    }
    return exp_nonpos(r.e - lD - q);
  }
};

// Energies from the bias model in FP32 (expanded form in log2 units, as in
// the FP32 on-the-fly sweeps); cf holds [A_col | A_st | B | C].
template <int D>
struct SrcModel32 {
  const float* xf;
  const float* cf;
  int K;
  struct Row {
    float a, b[D], c[D];
  };
  __device__ Row row(int k, double) const {
    Row r;
    r.a = cf[K + k];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      r.b[j] = cf[2 * K + (int64_t)j * K + k];
      r.c[j] = cf[2 * K + (int64_t)(D + j) * K + k];
    }
    return r;
  }
  __device__ double col(int64_t n, const double* logD) const { return -1.4426950408889634 * logD[n]; }
  __device__ double p(const Row& r, int64_t n, double e) const {
    float v = r.a + (float)e;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const float x = xf[n * D + j];
      v = __builtin_fmaf(r.b[j], x, v);
      v = __builtin_fmaf(r.c[j], x * x, v);
    }
    return (double)__builtin_amdgcn_exp2f(v);
  }
};

template <class Src>
__global__ void __launch_bounds__(256)
    hessian_partial_kernel(Src src, int K, int64_t N, const double* __restrict__ cst,
                           const double* __restrict__ gk, const double* __restrict__ logD,
                           int nb, int chunks, int64_t chunk_len, double* __restrict__ partials) {
  __shared__ double Pi[HB][HP];
  __shared__ double Pj[HB][HP];
  const int blk = blockIdx.x / chunks;
  const int chunk = blockIdx.x % chunks;
  int bi, bj;
  block_coords(blk, nb, bi, bj);
  const bool diag = (bi == bj);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;

  // loader mapping: row r = tid / 4, samples (tid % 4) * 4 .. + 3
  const int lr = tid >> 2;
  const int ls = (tid & 3) * 4;
  const int ki = bi * HB + lr;
  const int kj = bj * HB + lr;
  const bool si = (ki < K) && gk[ki] != 0.0;
  const bool sj = (kj < K) && gk[kj] != 0.0;
  const typename Src::Row ri = src.row(si ? ki : 0, si ? cst[ki] : 0.0);
  const typename Src::Row rj = src.row(sj ? kj : 0, sj ? cst[kj] : 0.0);

  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (d4){0.0, 0.0, 0.0, 0.0};

  const int64_t n_begin = (int64_t)chunk * chunk_len;
  int64_t n_end = n_begin + chunk_len;
  if (n_end > N) n_end = N;

  for (int64_t n0 = n_begin; n0 < n_end; n0 += HS) {
    // form P for the two slabs
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t n = n0 + ls + q;
      const bool ok = n < n_end;
      const double lD = ok ? src.col(n, logD) : 0.0;
      Pi[lr][ls + q] = (si && ok) ? src.p(ri, n, lD) : 0.0;
      if (!diag) Pj[lr][ls + q] = (sj && ok) ? src.p(rj, n, lD) : 0.0;
    }
    __syncthreads();
    const double(*Bsrc)[HP] = diag ? Pi : Pj;
#pragma unroll
    for (int s = 0; s < HS / 4; ++s) {
      const int col = s * 4 + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = Pi[wi * 32 + a * 16 + (lane & 15)][col];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bsrc[wj * 32 + b * 16 + (lane & 15)][col];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  // write the partial block: in the 16 x 16 FP64 accumulator, lane l holds
  // element v (0..3) at row l/16 + 4 v, column l % 16 of each tile
  double* out = partials + (int64_t)blockIdx.x * HB * HB;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wi * 32 + a * 16 + (lane >> 4) + 4 * v;
        const int c = wj * 32 + b * 16 + (lane & 15);
        out[r * HB + c] = acc[a][b][v];
      }
}

// ---- K <= 256: one workgroup per chunk of samples covers every state -------
//
// Per step of 16 samples the workgroup forms P for all K_pad = 16 ceil(K/16)
// rows once (one exponential per element, rows of 16 samples read as four
// 32-byte runs) into LDS, then its waves accumulate the upper-triangle 16 x 16
// tiles of G = P P^T, tile t going to wave t % NW (TPW tiles per wave, FP64
// accumulators in registers). Each chunk writes its K_pad x K_pad partial
// (upper tiles) for the fixed-order reduction.
constexpr int kSmallMaxK = 256;

// Sources with a two-stage p (load, then fin) take the software-pipelined loop.
template <class S, class = void>
struct SplitSource : std::false_type {};
template <class S>
struct SplitSource<S, std::void_t<decltype(&S::load)>> : std::true_type {};

template <class Src, int NW, int TPW>
__global__ void __launch_bounds__(NW * 64)
    hessian_small_kernel(Src src, int K, int Kp, int64_t N, const double* __restrict__ cst,
                         const double* __restrict__ gk, const double* __restrict__ logD,
                         int64_t chunk_len, double* __restrict__ partials) {
  constexpr int NT = NW * 64;
  constexpr int RPP = NT / 4;  // rows per loader pass
  __shared__ double P[kSmallMaxK][HP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int T = Kp / 16;
  const int ntiles = T * (T + 1) / 2;
  // tiles of this wave: t = wave + j NW -> (ti, tj), ti <= tj, row-major
  int ti[TPW], tj[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    int t = wave + j * NW, a = 0;
    if (t >= ntiles) t = -1;
    if (t >= 0)
      while (t >= T - a) {
        t -= T - a;
        ++a;
      }
    ti[j] = t >= 0 ? a : -1;
    tj[j] = t >= 0 ? a + t : -1;
  }
  // loader rows of this thread: r = tid / 4 + pass * RPP
  const int lr = tid >> 2;
  const int ls = (tid & 3) * 4;
  constexpr int MAXP = kSmallMaxK / RPP;
  typename Src::Row rows[MAXP];
  bool live[MAXP];
#pragma unroll
  for (int q = 0; q < MAXP; ++q) {
    const int k = lr + q * RPP;
    live[q] = k < K && gk[k] != 0.0;
    rows[q] = src.row(live[q] ? k : 0, live[q] ? cst[k] : 0.0);
  }
  d4 acc[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) acc[j] = (d4){0.0, 0.0, 0.0, 0.0};

  const int64_t n_begin = (int64_t)blockIdx.x * chunk_len;
  int64_t n_end = n_begin + chunk_len;
  if (n_end > N) n_end = N;
  // the MFMAs of one step of HS samples (P in LDS)
  auto mfma_step = [&]() {
#pragma unroll
    for (int sidx = 0; sidx < HS / 4; ++sidx) {
      const int c = sidx * 4 + (lane >> 4);
#pragma unroll
      for (int j = 0; j < TPW; ++j) {
        if (ti[j] < 0) continue;  // uniform per wave
        const double av = P[ti[j] * 16 + (lane & 15)][c];
        const double bv = P[tj[j] * 16 + (lane & 15)][c];
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[j], 0, 0, 0);
      }
    }
  };
  // (the 8-wave shapes of the FP64 / FP32 matrix sources would spill with
  // the extra registers, so they keep the plain loop)
  constexpr bool kPipe =
      SplitSource<Src>::value && (NW == 4 || std::is_same<Src, SrcMatExp32>::value);
  if constexpr (kPipe) {
    // software pipeline: the loads of step t + 1 are issued before the MFMAs
    // of step t and consumed after them (clamped addresses, so every load is
    // in bounds; rows without samples load row 0 and are zeroed)
    using Raw = typename Src::Raw;
    double cv[4];
    Raw uv[MAXP][4];
    auto fetch = [&](int64_t n0) {
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int64_t n = n0 + ls + w < n_end ? n0 + ls + w : n_end - 1;
        cv[w] = src.col(n, logD);
#pragma unroll
        for (int q = 0; q < MAXP; ++q)
          if (lr + q * RPP < Kp) uv[q][w] = src.load(rows[q], n);
      }
    };
    if (n_begin < n_end) fetch(n_begin);
    for (int64_t n0 = n_begin; n0 < n_end; n0 += HS) {
#pragma unroll
      for (int q = 0; q < MAXP; ++q) {
        const int r = lr + q * RPP;
        if (r < Kp) {
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int64_t n = n0 + ls + w;
            P[r][ls + w] = (live[q] && n < n_end) ? src.fin(rows[q], uv[q][w], cv[w]) : 0.0;
          }
        }
      }
      __syncthreads();
      if (n0 + HS < n_end) fetch(n0 + HS);
      mfma_step();
      __syncthreads();
    }
  } else {
    for (int64_t n0 = n_begin; n0 < n_end; n0 += HS) {
      double col[4];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int64_t n = n0 + ls + w;
        col[w] = n < n_end ? src.col(n, logD) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < MAXP; ++q) {
        const int r = lr + q * RPP;
        if (r < Kp) {
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int64_t n = n0 + ls + w;
            P[r][ls + w] = (live[q] && n < n_end) ? src.p(rows[q], n, col[w]) : 0.0;
          }
        }
      }
      __syncthreads();
      mfma_step();
      __syncthreads();
    }
  }
  // lane l holds element v at row l/16 + 4 v, column l % 16 of each tile
  double* out = partials + (int64_t)blockIdx.x * Kp * Kp;
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    if (ti[j] < 0) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = ti[j] * 16 + (lane >> 4) + 4 * v;
      const int c = tj[j] * 16 + (lane & 15);
      out[(int64_t)r * Kp + c] = acc[j][v];
    }
  }
}

// H_ij = delta_ij S_i - sum_chunks G_ij for i <= j (upper tiles), mirrored.
__global__ void __launch_bounds__(256)
    hessian_small_reduce_kernel(int K, int Kp, int chunks, const double* __restrict__ partials,
                                const double* __restrict__ S, const double* __restrict__ gk,
                                double* __restrict__ H) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)K * K) return;
  const int i = (int)(e / K), j = (int)(e % K);
  if (j < i) return;
  // the partial holds the upper tiles: (i, j) lies in tile (i/16, j/16) with
  // i/16 <= j/16 since i <= j
  double g = 0.0;
  const double* p = partials + (int64_t)i * Kp + j;
  for (int q = 0; q < chunks; ++q) g += p[(int64_t)q * Kp * Kp];
  double v = -g;
  if (i == j) v += (gk[i] != 0.0) ? S[i] : 0.0;
  if (gk[i] == 0.0 || gk[j] == 0.0) v = 0.0;
  H[(int64_t)i * K + j] = v;
  H[(int64_t)j * K + i] = v;
}

static int small_kp(int K) { return (K + 15) / 16 * 16; }

static int small_chunks(int64_t N, int num_cus) {
  int64_t g = 2 * (int64_t)num_cus;
  const int64_t by_n = (N + 255) / 256;  // at least 256 samples per chunk
  if (g > by_n) g = by_n;
  return (int)(g < 1 ? 1 : g);
}

// ---- mixed precision, K > 256: FP16 matrix cores ----------------------------
//
// The Hessian only shapes the Newton steps (the fixed point is set by the
// FP64 gradient), so for K > 256 P is formed in FP32 (exp2 of an exponent in
// log2 units), rounded to FP16 (P_kn lies in [0, 1]: sum_k P_kn = 1), and
// G = P P^T runs on v_mfma_f32_16x16x32_f16 with FP32 accumulation inside a
// sample chunk and FP64 across chunks.
//
// P is materialised once per Hessian: forming it inside the product would
// recompute every exponential for each 256-row block a state belongs to
// (7.8 times over at K = 1600), which left the matrix cores idle behind the
// VALU. The FP16 copy is sample-tiled: tile t holds samples 32 t .. 32 t + 31
// of every state, state k at (t K + k) 32 halves, so the 256-row slab of a
// block at one tile is a contiguous 16 KB run. At most 4 GiB of it is held;
// longer problems are filled and multiplied super-chunk by super-chunk, the
// product adding into the same partial blocks.
//
// Product: a workgroup (8 waves) owns one 256 x 256 output block (bi <= bj)
// and one chunk of tiles. Per tile it copies the two slabs into LDS, 1 KB
// per wave instruction, and wave w accumulates the 64 x 128 output tile (rows
// 64 (w % 4), columns 128 (w / 4)) as 4 x 8 MFMA tiles. LDS is
// double-buffered (the next tile's loads are in flight during the matrix
// instructions), one barrier per tile. The hardware deals workgroups to the
// 8 XCDs round robin; the grid is ordered so that the workgroups one XCD
// runs together are all block pairs of one sample chunk, which share the
// slabs in that XCD's L2 instead of each pulling them from HBM, and every
// block pair does the same work so that they stay in step.
// Operand layout (checked on the hardware): A lane l holds row l % 16,
// k = 8 (l / 16) .. + 7; B lane l holds column l % 16, the same k; the
// accumulator lane l holds rows 4 (l / 16) + i, column l % 16.
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int XB = 256;      // output block edge
constexpr int XS = 32;       // samples per tile (one MFMA k-extent)
constexpr int XP = XS + 8;   // padded LDS row (halves): rows 80 bytes apart
constexpr double kLog2eH = 1.4426950408889634;
constexpr int64_t kP16Bytes = int64_t(1) << 32;  // cap of the FP16 copy of P

// Per-sample column constant in log2 units, once per Hessian:
// c_n = -log2(e) ln D_n.
__global__ void __launch_bounds__(256)
    h16_colv_kernel(int64_t N, const double* __restrict__ logD, float* __restrict__ colv) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  colv[n] = (float)(-kLog2eH * logD[n]);
}

// Exponents t_kn (log2 units) of 16 consecutive samples n .. n + 15 of one
// row: full() when all 16 lie before the end, tail() otherwise (indices
// clamped to the last sample; the caller zeroes those values).

// FP32 model (the log2-domain coefficients of the FP32 model sweeps):
// t_kn = A_k + e_n + sum_j x_nj (B_jk + C_jk x_nj), e_n = -log2(e) ln D_n.
template <int D>
struct SrcModel32f {
  const float* xf;
  const float* cf;
  int K;
  struct Row {
    float a, b[D], c[D];
  };
  __device__ Row row(int k) const {
    Row rw;
    rw.a = cf[K + k];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      rw.b[j] = cf[2 * K + (int64_t)j * K + k];
      rw.c[j] = cf[2 * K + (int64_t)(D + j) * K + k];
    }
    return rw;
  }
  __device__ float eval(const Row& rw, float e, const float* x) const {
    float v = rw.a + e;
#pragma unroll
    for (int j = 0; j < D; ++j) v = __builtin_fmaf(__builtin_fmaf(rw.c[j], x[j], rw.b[j]), x[j], v);
    return v;
  }
  __device__ void full(const Row& rw, int64_t n, const float* __restrict__ colv,
                       float (&t)[16]) const {
#pragma unroll
    for (int h = 0; h < 16; h += 8) {
      float cv[8], x[8 * D];
#pragma unroll
      for (int q = 0; q < 8; ++q) cv[q] = colv[n + h + q];
#pragma unroll
      for (int i = 0; i < 8 * D; ++i) x[i] = xf[(n + h) * D + i];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[h + q] = eval(rw, cv[q], &x[q * D]);
    }
  }
  __device__ void tail(const Row& rw, int64_t n, int64_t last, const float* __restrict__ colv,
                       float (&t)[16]) const {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int64_t m = n + q < last ? n + q : last;
      float x[D];
#pragma unroll
      for (int j = 0; j < D; ++j) x[j] = xf[m * D + j];
      t[q] = eval(rw, colv[m], x);
    }
  }
};

// Model fill: a wave takes 64 states of one tile (32 samples per lane), so
// the per-sample coordinates and column constants are wave-uniform scalar
// loads and each element costs the expanded quadratic, one exp2 and a
// conversion. Kr = K rounded up to 64. Samples [n_begin, n_end) as tiles
// 0 .. nt - 1; past n_end the copy is 0, and so are the rows of unsampled
// states.
template <int D>
__global__ void __launch_bounds__(256)
    p16t_fill_model_kernel(SrcModel32f<D> src, int K, int Kr, int64_t n_begin, int64_t n_end,
                           int64_t nt, const double* __restrict__ gk,
                           const float* __restrict__ colv, _Float16* __restrict__ P) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t t = __builtin_amdgcn_readfirstlane((int)(e / Kr));
  if (t >= nt) return;
  const int k = (int)(e - t * Kr);
  if (k >= K) return;
  const bool on = gk[k] != 0.0;
  const typename SrcModel32f<D>::Row rw = src.row(k);
  const int64_t n0 = n_begin + t * XS;
  const bool whole = n0 + XS <= n_end;
  _Float16* dst = P + (t * K + k) * XS;
#pragma unroll
  for (int h = 0; h < XS; h += 8) {
    h8v v;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t n = n0 + h + j;
      const int64_t m = whole || n < n_end ? n : n_end - 1;
      float x[D];
#pragma unroll
      for (int i = 0; i < D; ++i) x[i] = src.xf[m * D + i];
      const float y = src.eval(rw, colv[m], x);
      v[j] = (_Float16)((on && (whole || n < n_end)) ? __builtin_amdgcn_exp2f(y) : 0.f);
    }
    *reinterpret_cast<h8v*>(dst + h) = v;
  }
}

// Stored FP64 or FP32 u: P_kn = fp16(exp2(fp32(log2(e) (c_k - u_kn)) + e_n)),
// the difference taken in FP64. A workgroup (4 waves) converts 16 states x
// 256 samples (8 tiles): each wave reads its 4 rows along n (16 bytes per
// lane, 1 KB of one row per instruction), forms the values in registers,
// transposes them through LDS, and the workgroup writes each tile's 16 rows
// as one 1 KB run. vec: rows 16-byte aligned (else element loads).
template <typename TI>
__global__ void __launch_bounds__(256)
    p16t_fill_stored_kernel(const TI* __restrict__ u, int64_t ld, bool vec, int K,
                            int64_t n_begin, int64_t n_end, int64_t nt,
                            const double* __restrict__ cst, const double* __restrict__ gk,
                            const float* __restrict__ colv, _Float16* __restrict__ P) {
  constexpr int R = 16, C = 256, CP = C + 8;
  constexpr int V = 16 / (int)sizeof(TI);  // elements per 16-byte load
  constexpr int NI = C / (64 * V);         // loads per row
  __shared__ __attribute__((aligned(16))) _Float16 T[R][CP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k0 = blockIdx.y * R;
  const int64_t s0 = n_begin + (int64_t)blockIdx.x * C;  // first sample of the block
  // all loads of the wave's 4 rows first (they are in flight together), then
  // the arithmetic
  TI x[4][NI][V];
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int k = k0 + wave * 4 + rr;
    const bool on = k < K;
    const TI* row = u + (int64_t)(on ? k : 0) * ld;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int64_t n = s0 + (i * 64 + lane) * V;
      if (on && vec && n + V <= n_end) {
        if constexpr (V == 2) {
          const double2 w = *reinterpret_cast<const double2*>(row + n);
          x[rr][i][0] = w.x;
          x[rr][i][1] = w.y;
        } else {
          const float4 w = *reinterpret_cast<const float4*>(row + n);
          x[rr][i][0] = w.x;
          x[rr][i][1] = w.y;
          x[rr][i][2] = w.z;
          x[rr][i][3] = w.w;
        }
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j) x[rr][i][j] = (on && n + j < n_end) ? row[n + j] : (TI)0;
      }
    }
  }
#pragma unroll
  for (int rr = 0; rr < 4; ++rr) {
    const int r = wave * 4 + rr;
    const int k = k0 + r;
    const bool on = k < K && gk[k] != 0.0;
    const double c = on ? cst[k] : 0.0;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int s = (i * 64 + lane) * V;  // sample within the block
      const int64_t n = s0 + s;
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const bool ok = on && n + j < n_end;
        const float cv = ok ? colv[n + j] : 0.f;
        T[r][s + j] = (_Float16)(
            ok ? __builtin_amdgcn_exp2f((float)(kLog2eH * (c - (double)x[rr][i][j])) + cv) : 0.f);
      }
    }
  }
  __syncthreads();
  // tile tl (0..7) of the block, row r, 16-sample half hf: 32 bytes per thread
  const int tl = threadIdx.x >> 5, r = (threadIdx.x >> 1) & 15, hf = threadIdx.x & 1;
  const int64_t t = (int64_t)blockIdx.x * (C / XS) + tl;
  const int k = k0 + r;
  if (t >= nt || k >= K) return;
  const h8v lo = *reinterpret_cast<const h8v*>(&T[r][tl * XS + hf * 16]);
  const h8v hi = *reinterpret_cast<const h8v*>(&T[r][tl * XS + hf * 16 + 8]);
  _Float16* dst = P + (t * K + k) * XS + hf * 16;
  *reinterpret_cast<h8v*>(dst) = lo;
  *reinterpret_cast<h8v*>(dst + 8) = hi;
}

// G over the tiles of one super-chunk; see the section comment. partials:
// one 256 x 256 FP32 block per (block pair, chunk), written (accumulate
// false) or added to.
__global__ void __launch_bounds__(512)
    hessian_p16t_kernel(const _Float16* __restrict__ P, int K, int64_t nt, int nb, int nblk,
                        int chunks, int64_t per, bool accumulate, float* __restrict__ partials) {
  __shared__ __attribute__((aligned(16))) _Float16 L[2][2][XB][XP];  // [buffer][slab][row][sample]
  const int wg = blockIdx.x;
  const int xcd = wg & 7, slot = wg >> 3;
  const int chunk = (slot / nblk) * 8 + xcd;
  const int blk = slot % nblk;
  int bi, bj;
  block_coords(blk, nb, bi, bj);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // copy role: 16-byte piece c = tid + 512 j of the tile's slabs (slab j / 2,
  // row (c % 1024) / 4, quarter c % 4). Every block pair does the same work:
  // a diagonal block copies its slab twice and the tiles past K are
  // multiplied (as zeros). Workgroups of one chunk then stay in step and
  // share each slab in their XCD's L2; with the shortcuts the faster ones ran
  // ahead and the slabs were fetched again from HBM (9% slower at K = 1600
  // despite 20% fewer MFMAs, the same at K = 1000).
  const int crow = (tid & 1023) >> 2, cq = tid & 3;
  // product role: output rows 64 wr + 16 a, columns 128 wc + 16 b
  const int wr = wave & 3, wc = wave >> 2;
  const int kq = (lane >> 4) * 8;
  f4v acc[4][8];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = (f4v){0.f, 0.f, 0.f, 0.f};

  const int64_t t_begin = (int64_t)chunk * per;
  const int64_t t_end = t_begin + per < nt ? t_begin + per : nt;
  h8v v[4];
  auto load = [&](int64_t t) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = ((j >> 1) ? bj : bi) * XB + crow + (j & 1) * 128;
      v[j] = (h8v){};
      if (k < K) v[j] = *reinterpret_cast<const h8v*>(P + (t * K + k) * XS + cq * 8);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      *reinterpret_cast<h8v*>(&L[buf][j >> 1][crow + (j & 1) * 128][cq * 8]) = v[j];
  };
  if (t_begin < t_end) {
    load(t_begin);
    store(0);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t t = t_begin; t < t_end; ++t) {
    const bool more = t + 1 < t_end;
    if (more) load(t + 1);
    const _Float16(*Pa)[XP] = L[cur][0];
    const _Float16(*Pb)[XP] = L[cur][1];
    h8v av[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
      av[a] = *reinterpret_cast<const h8v*>(&Pa[wr * 64 + a * 16 + (lane & 15)][kq]);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const h8v bv = *reinterpret_cast<const h8v*>(&Pb[wc * 128 + b * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int a = 0; a < 4; ++a)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av[a], bv, acc[a][b], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  float* out = partials + ((int64_t)blk * chunks + chunk) * XB * XB;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = wr * 64 + a * 16 + (lane >> 4) * 4 + q;
        const int c = wc * 128 + b * 16 + (lane & 15);
        if (accumulate)
          out[r * XB + c] += acc[a][b][q];
        else
          out[r * XB + c] = acc[a][b][q];
      }
}

// H_ij = delta_ij S_i - sum_chunks G_ij (FP64 sum in a fixed order), both triangles.
__global__ void __launch_bounds__(256)
    hessian_h16_reduce_kernel(int K, int nb, int chunks, const float* __restrict__ partials,
                              const double* __restrict__ S, const double* __restrict__ gk,
                              double* __restrict__ H) {
  const int blk = blockIdx.y;
  int bi, bj;
  block_coords(blk, nb, bi, bj);
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= XB * XB) return;
  const int r = e / XB, c = e % XB;
  const int i = bi * XB + r, j = bj * XB + c;
  if (i >= K || j >= K) return;
  if (bi == bj && j < i) return;
  double g = 0.0;
  const float* p = partials + ((int64_t)blk * chunks) * XB * XB + e;
  for (int q = 0; q < chunks; ++q) g += (double)p[(int64_t)q * XB * XB];
  double v = -g;
  if (i == j) v += (gk[i] != 0.0) ? S[i] : 0.0;
  if (gk[i] == 0.0 || gk[j] == 0.0) v = 0.0;
  H[(int64_t)i * K + j] = v;
  H[(int64_t)j * K + i] = v;
}

static int h16_nb(int K) { return (K + XB - 1) / XB; }

int64_t p16_samples(int K, int64_t N) {
  // whole tiles, at most kP16Bytes of FP16 (K halves per sample)
  const int64_t all = (N + XS - 1) / XS * XS;
  int64_t cap = kP16Bytes / (2 * (int64_t)K) / XS * XS;
  if (cap < XS) cap = XS;
  return all < cap ? all : cap;
}

static int h16_chunks(int K, int64_t N, int num_cus) {
  // chunks = 8 m (the XCD-ordered grid takes a multiple of 8): per XCD the
  // nblk m workgroups run on num_cus / 8 CUs, one each at a time; pick the m
  // in [1, 16] whose last round is fullest (ties: fewer chunks), each chunk at
  // least 16 tiles of the super-chunk
  const int nb = h16_nb(K);
  const int nblk = nb * (nb + 1) / 2;
  const int per_xcd = num_cus / 8 > 0 ? num_cus / 8 : 1;
  const int64_t tiles = p16_samples(K, N) / XS;
  int64_t m_max = tiles / (8 * 16);
  if (m_max > 16) m_max = 16;
  if (m_max < 1) m_max = 1;
  int best = 1;
  double best_eff = 0.0;
  for (int m = 1; m <= m_max; ++m) {
    const int64_t wgs = (int64_t)nblk * m;
    const int64_t rounds = (wgs + per_xcd - 1) / per_xcd;
    const double eff = (double)wgs / (double)(rounds * per_xcd);
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = m;
    }
  }
  return 8 * best;
}

// H_ij = delta_ij S_i - sum_chunks G_ij, written to both triangles.
__global__ void __launch_bounds__(256)
    hessian_reduce_kernel(int K, int nb, int chunks, const double* __restrict__ partials,
                          const double* __restrict__ S, const double* __restrict__ gk,
                          double* __restrict__ H) {
  const int blk = blockIdx.y;
  int bi, bj;
  block_coords(blk, nb, bi, bj);
  const int e = blockIdx.x * 256 + threadIdx.x;  // element in the 64 x 64 block
  if (e >= HB * HB) return;
  const int r = e / HB, c = e % HB;
  const int i = bi * HB + r, j = bj * HB + c;
  if (i >= K || j >= K) return;
  if (bi == bj && j < i) return;  // lower half of a diagonal block: mirror of the upper
  double g = 0.0;
  const double* p = partials + ((int64_t)blk * chunks) * HB * HB + e;
  for (int q = 0; q < chunks; ++q) g += p[(int64_t)q * HB * HB];
  double v = -g;
  if (i == j) v += (gk[i] != 0.0) ? S[i] : 0.0;
  if (gk[i] == 0.0 || gk[j] == 0.0) v = 0.0;
  H[(int64_t)i * K + j] = v;
  H[(int64_t)j * K + i] = v;
}

static int hess_nb(int K) { return (K + HB - 1) / HB; }

size_t hessian_partial_count(int K, int64_t N, int num_cus, int* chunks_out) {
  if (K <= kSmallMaxK) {
    const int ch = small_chunks(N, num_cus);
    if (chunks_out) *chunks_out = ch;
    const size_t kp = (size_t)small_kp(K);
    return (size_t)ch * kp * kp;
  }
  const int nb = hess_nb(K);
  const int nblk = nb * (nb + 1) / 2;
  // aim for about 4 workgroups per CU, each chunk at least 256 samples
  int chunks = (4 * num_cus + nblk - 1) / nblk;
  const int64_t max_chunks = (N + 255) / 256;
  if (chunks > max_chunks) chunks = (int)max_chunks;
  if (chunks < 1) chunks = 1;
  if (chunks_out) *chunks_out = chunks;
  // room for the FP16-core path of the mixed-precision sources as well
  // (FP32 partial blocks, then the N per-sample column constants)
  const int nb16 = h16_nb(K);
  const size_t h16 =
      (size_t)(nb16 * (nb16 + 1) / 2) * h16_chunks(K, N, num_cus) * XB * XB + (size_t)N + 64;
  const size_t fp64 = (size_t)nblk * chunks * HB * HB;
  return fp64 > (h16 + 1) / 2 ? fp64 : (h16 + 1) / 2;
}

template <class Src>
static void launch_partial(hipStream_t s, const Src& src, int K, int64_t N, const double* cst,
                           const double* gk, const double* logD, int nb, int chunks,
                           int64_t chunk_len, double* partials) {
  const int nblk = nb * (nb + 1) / 2;
  hipLaunchKernelGGL(hessian_partial_kernel<Src>, dim3(nblk * chunks), dim3(256), 0, s, src, K, N,
                     cst, gk, logD, nb, chunks, chunk_len, partials);
}

template <class Src>
static void launch_small(hipStream_t s, const Src& src, int K, int64_t N, const double* cst,
                         const double* gk, const double* logD, int chunks, double* partials) {
  const int Kp = small_kp(K);
  int64_t chunk_len = (N + chunks - 1) / chunks;
  chunk_len = (chunk_len + HS - 1) / HS * HS;
  const int T = Kp / 16, nt = T * (T + 1) / 2;
  // 4 waves up to 36 tiles (K <= 128), else 8 waves (up to 136 tiles)
  if (nt <= 4 * 9)
    hipLaunchKernelGGL((hessian_small_kernel<Src, 4, 9>), dim3(chunks), dim3(256), 0, s, src, K, Kp,
                       N, cst, gk, logD, chunk_len, partials);
  else
    hipLaunchKernelGGL((hessian_small_kernel<Src, 8, 17>), dim3(chunks), dim3(512), 0, s, src, K,
                       Kp, N, cst, gk, logD, chunk_len, partials);
}

template <class Src>
static void launch_any(hipStream_t s, const Src& src, int K, int64_t N, const double* cst,
                       const double* gk, const double* logD, int nb, int chunks,
                       int64_t chunk_len, double* partials) {
  if (K <= kSmallMaxK)
    launch_small(s, src, K, N, cst, gk, logD, chunks, partials);
  else
    launch_partial(s, src, K, N, cst, gk, logD, nb, chunks, chunk_len, partials);
}

hipError_t launch_hessian(hipStream_t s, const HessSource& hs, int K, int64_t N,
                          const double* cst, const double* gk, const double* logD,
                          const double* S, double* partials, int chunks, double* H) {
  const int nb = hess_nb(K);
  const int nblk = nb * (nb + 1) / 2;
  int64_t chunk_len = (N + chunks - 1) / chunks;
  chunk_len = (chunk_len + HS - 1) / HS * HS;
  if (K > kSmallMaxK && (hs.kind == 3 || hs.kind == 5 || hs.kind == 8)) {
    // P once into the tiled FP16 copy (per super-chunk), then the product
    if (!hs.p16) return hipErrorInvalidValue;
    const int nb16 = h16_nb(K);
    const int nblk16 = nb16 * (nb16 + 1) / 2;
    const int ch16 = h16_chunks(K, N, hs.num_cus);
    const int64_t len = p16_samples(K, N);
    float* p16 = reinterpret_cast<float*>(partials);
    float* colv = p16 + (size_t)nblk16 * ch16 * XB * XB;
    _Float16* P = reinterpret_cast<_Float16*>(hs.p16);
    hipLaunchKernelGGL(h16_colv_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N,
                       logD, colv);
    const int esz = hs.kind == 5 ? 8 : 4;
    const bool vec = hs.kind != 3 && (hs.ld % (16 / esz)) == 0 &&
                     (reinterpret_cast<uintptr_t>(hs.u) & 15) == 0;
    for (int64_t n0 = 0; n0 < N; n0 += len) {
      const int64_t n1 = n0 + len < N ? n0 + len : N;
      const int64_t nt = (n1 - n0 + XS - 1) / XS;
      if (hs.kind == 3) {
        const int Kr = (K + 63) / 64 * 64;
        const int64_t tot = nt * Kr;
        const dim3 gf((unsigned)((tot + 255) / 256));
        if (hs.otf.d == 1)
          hipLaunchKernelGGL(p16t_fill_model_kernel<1>, gf, dim3(256), 0, s,
                             SrcModel32f<1>{hs.otf.xf, hs.otf.cf32, K}, K, Kr, n0, n1, nt, gk, colv,
                             P);
        else
          hipLaunchKernelGGL(p16t_fill_model_kernel<2>, gf, dim3(256), 0, s,
                             SrcModel32f<2>{hs.otf.xf, hs.otf.cf32, K}, K, Kr, n0, n1, nt, gk, colv,
                             P);
      } else {
        const dim3 gf((unsigned)((nt + 7) / 8), (unsigned)((K + 15) / 16));
        if (hs.kind == 5)
          hipLaunchKernelGGL(p16t_fill_stored_kernel<double>, gf, dim3(256), 0, s,
                             reinterpret_cast<const double*>(hs.u), hs.ld, vec, K, n0, n1, nt,
                             cst, gk, colv, P);
        else
          hipLaunchKernelGGL(p16t_fill_stored_kernel<float>, gf, dim3(256), 0, s,
                             reinterpret_cast<const float*>(hs.u), hs.ld, vec, K, n0, n1, nt,
                             cst, gk, colv, P);
      }
      const int64_t per = (nt + ch16 - 1) / ch16;
      hipLaunchKernelGGL(hessian_p16t_kernel, dim3(nblk16 * ch16), dim3(512), 0, s, P, K, nt,
                         nb16, nblk16, ch16, per, n0 > 0, p16);
    }
    hipLaunchKernelGGL(hessian_h16_reduce_kernel, dim3(XB * XB / 256, nblk16), dim3(256), 0, s, K,
                       nb16, ch16, p16, S, gk, H);
    return hipGetLastError();
  }
  switch (hs.kind) {
    case 0:
    case 5:  // FP64 u where the FP16-core path does not apply (K <= kSmallMaxK)
      launch_any(s, SrcMat<double>{reinterpret_cast<const double*>(hs.u), hs.ld}, K, N, cst,
                     gk, logD, nb, chunks, chunk_len, partials);
      break;
    case 6:
      launch_any(s, SrcMatExp32{reinterpret_cast<const double*>(hs.u), hs.ld}, K, N, cst, gk,
                     logD, nb, chunks, chunk_len, partials);
      break;
    case 1:
    case 8:  // FP32 u where the FP16-core path does not apply (K <= kSmallMaxK)
      launch_any(s, SrcMat<float>{reinterpret_cast<const float*>(hs.u), hs.ld}, K, N, cst, gk,
                     logD, nb, chunks, chunk_len, partials);
      break;
    case 2:
      launch_any(s, SrcPacked{reinterpret_cast<const float*>(hs.u), hs.ld, hs.m0}, K, N, cst,
                     gk, logD, nb, chunks, chunk_len, partials);
      break;
    case 3:
      if (hs.otf.d == 1)
        launch_any(s, SrcModel32<1>{hs.otf.xf, hs.otf.cf32, K}, K, N, cst, gk, logD, nb, chunks,
                       chunk_len, partials);
      else
        launch_any(s, SrcModel32<2>{hs.otf.xf, hs.otf.cf32, K}, K, N, cst, gk, logD, nb, chunks,
                       chunk_len, partials);
      break;
    default:
      if (hs.otf.model == BUMBAR_MODEL_HARMONIC) {
        if (hs.otf.d == 1)
          launch_any(s, SrcModel64<1, BUMBAR_MODEL_HARMONIC>{hs.otf.xi, hs.otf.cf64, K}, K, N,
                         cst, gk, logD, nb, chunks, chunk_len, partials);
        else
          launch_any(s, SrcModel64<2, BUMBAR_MODEL_HARMONIC>{hs.otf.xi, hs.otf.cf64, K}, K, N,
                         cst, gk, logD, nb, chunks, chunk_len, partials);
      } else {
        if (hs.otf.d == 1)
          launch_any(s, SrcModel64<1, BUMBAR_MODEL_LINEAR>{hs.otf.xi, hs.otf.cf64, K}, K, N,
                         cst, gk, logD, nb, chunks, chunk_len, partials);
        else
          launch_any(s, SrcModel64<2, BUMBAR_MODEL_LINEAR>{hs.otf.xi, hs.otf.cf64, K}, K, N,
                         cst, gk, logD, nb, chunks, chunk_len, partials);
      }
  }
  if (K <= kSmallMaxK)
    hipLaunchKernelGGL(hessian_small_reduce_kernel, dim3((unsigned)(((int64_t)K * K + 255) / 256)),
                       dim3(256), 0, s, K, small_kp(K), chunks, partials, S, gk, H);
  else
    hipLaunchKernelGGL(hessian_reduce_kernel, dim3(HB * HB / 256, nblk), dim3(256), 0, s, K, nb,
                       chunks, partials, S, gk, H);
  return hipGetLastError();
}

}  // namespace bumbar
