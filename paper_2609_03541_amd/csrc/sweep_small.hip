// Batches of self-consistent steps (Eq. (1), with the bin multiplicities h_n
// of the binned stage, Algorithm 1) on a level small enough for one
// workgroup. The first level of the binned stage has a few hundred bins at
// most and takes most of the stage's steps; as separate sweep and finaliser
// launches every such step is bound by launch and memory latency (a few
// thousand exponentials spread over two workgroups). Here the K x P matrix is
// loaded once into registers and a whole batch of steps runs between
// workgroup barriers: per step a column pass (max, shifted exponentials,
// ln D_n), a per-state pass through LDS, and the finalisation (new f, the
// gauge f_0 = 0, the relative step of Eq. (2) and the other scalars).
//
// Each step writes what a sweep followed by its finaliser writes: f_new to
// its slot of the history, its scalars (flags included, so that the caller's
// fallback to the robust sweep is unchanged), ln D_n, ln S_k and S_k; after
// the batch the constants c_k = ln N'_k + f_k, the sampled flags and ln N'_k
// are left as the next sweep expects them. All sums run in a fixed order, so
// the results do not depend on timing.
//
// The fused kernels run the batches of several independent problems (a
// serving mix) together: a fixed grid walks a device work list, each
// workgroup running whole items with the same inlined code; one kernel per
// column layout present in the list.
#include <hip/hip_runtime.h>

#include <cmath>

#include "bumbar_impl.h"
#include "devmath.h"

namespace bumbar {

namespace {

constexpr int kSB = 1024;  // threads of the workgroup
constexpr int kSR = 16;    // states held per thread

// Thread (kr, nc) = (tid / NC, tid % NC) holds column nc and states
// kr, kr + KR, ..., so K <= KR * kSR and P <= NC.
template <int NC>
struct SmallShared {
  static constexpr int KR = kSB / NC;
  static constexpr int KC = KR * kSR;
  double sp[KC * (NC + 1)];  // per-state column terms, rows padded against bank conflicts
  double cm[KR * NC];        // column maxima per row group
  double ds[KR * NC];        // column sums per row group
  double wv[NC];             // h_n / D'_n
  double c[KC];              // c_k = ln N'_k + f_k
  double f[KC];              // current f
  double lnNp[KC];
  double nk[KC];             // N_k
  double fn[KC];             // unnormalised new f
  double red[kSB / 64][6];
  unsigned flags[2];
};

// The batch of one problem on the workgroup's LDS block L (every thread of
// the workgroup calls it).
template <int NC>
__device__ __forceinline__ void small_steps(SmallShared<NC>& L, const double* __restrict__ u,
                                            int64_t ld, int K, int P,
                                            const double* __restrict__ h,
                                            const int64_t* __restrict__ Nk,
                                            const double* __restrict__ f_in, int T,
                                            double* __restrict__ f_hist,
                                            SweepScalars* __restrict__ scal,
                                            double* __restrict__ logD,
                                            double* __restrict__ lnS_out,
                                            double* __restrict__ S_out,
                                            double* __restrict__ cst,
                                            double* __restrict__ gk_out,
                                            double* __restrict__ lnNp_out) {
  using SS = SmallShared<NC>;
  constexpr int KR = SS::KR;
  const int tid = threadIdx.x;
  const int nc = tid % NC, kr = tid / NC;
  const bool colv = nc < P;
  const int nrow = kr < K ? (K - 1 - kr) / KR + 1 : 0;
  double U[kSR];
#pragma unroll
  for (int j = 0; j < kSR; ++j)
    U[j] = (j < nrow && colv) ? u[(int64_t)(kr + KR * j) * ld + nc] : 0.0;
  const double hn = colv ? (h != nullptr ? h[nc] : 1.0) : 0.0;
  for (int k = tid; k < K; k += kSB) {
    const int64_t n = Nk[k];
    const double l = n > 0 ? log((double)n) : 0.0;
    L.lnNp[k] = l;
    L.nk[k] = (double)n;
    L.f[k] = f_in[k];
    L.c[k] = l + f_in[k];
  }
  if (tid == 0) L.flags[0] = 0u;
  // R consecutive lanes per state add that state's column terms
  int R = 1;
  while (R < 64 && 2 * R * K <= kSB && 2 * R <= NC) R *= 2;
  const int sk = tid / R, sr = tid % R;
  const bool owner = sr == 0 && sk < K;
  __syncthreads();
  unsigned smask = 0u;
#pragma unroll
  for (int j = 0; j < kSR; ++j)
    if (j < nrow && L.nk[kr + KR * j] > 0.0) smask |= 1u << j;

  for (int it = 0; it < T; ++it) {
    if (tid == 0) L.flags[(it + 1) & 1] = 0u;
    unsigned bad = 0u;
    // opaque per step: row addresses and row predicates are recomputed in
    // each step rather than hoisted out of the loop into registers
    int kro = kr, nro = nrow;
    unsigned smo = smask;
    asm volatile("" : "+v"(kro), "+v"(nro), "+v"(smo));
    // column pass: a = c - u and the maximum over all states
    double mx = -INFINITY, chk = 0.0;
#pragma unroll
    for (int j = 0; j < kSR; ++j) {
      if (j < nro) {
        const double a = L.c[kro + KR * j] - U[j];
        mx = fmax(mx, a);
        chk += a;
      }
    }
    if (colv && chk != chk) bad |= FLAG_NAN;
    L.cm[kr * NC + nc] = mx;
    __syncthreads();
    double m = L.cm[nc];
#pragma unroll
    for (int w = 1; w < KR; ++w) m = fmax(m, L.cm[w * NC + nc]);
    if (m == -INFINITY) m = 0.0;
    // shifted exponentials, kept in LDS; D' sums the sampled states
    double dsum = 0.0;
#pragma unroll
    for (int j = 0; j < kSR; ++j) {
      if (j < nro) {
        const double e = exp_nonpos(L.c[kro + KR * j] - U[j] - m);
        if ((smo >> j) & 1u) dsum += e;
        L.sp[(kro + KR * j) * (NC + 1) + nc] = e;
      }
      // four exponentials in flight at a time keep the registers in bounds
      if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    L.ds[kr * NC + nc] = dsum;
    __syncthreads();
    double obj = 0.0;
    if (kr == 0) {
      double D = L.ds[nc];
#pragma unroll
      for (int w = 1; w < KR; ++w) D += L.ds[w * NC + nc];
      double wn = 0.0;
      if (colv) {
        if (!(D >= 1e-300 && D <= 1e300)) bad |= FLAG_COL;
        wn = hn * rcp_nr(D);
        const double l = m + log(D);
        if (logD != nullptr) logD[nc] = l;
        obj = hn * l;
      }
      L.wv[nc] = wn;
    }
    __syncthreads();
    // per-state pass: S'_k = sum_n h_n exp(c_k - u_kn) / D_n
    double Sp = 0.0;
    if (sk < K) {
      const double* row = &L.sp[sk * (NC + 1)];
      double s0 = 0.0, s1 = 0.0;
      int i = sr;
      for (; i + R < P; i += 2 * R) {
        s0 = __builtin_fma(row[i], L.wv[i], s0);
        s1 = __builtin_fma(row[i + R], L.wv[i + R], s1);
      }
      if (i < P) s0 = __builtin_fma(row[i], L.wv[i], s0);
      Sp = s0 + s1;
    }
    for (int off = 1; off < R; off <<= 1) Sp += __shfl_xor(Sp, off, 64);
    double f_old = 0.0;
    if (owner) {
      f_old = L.f[sk];
      const double lnS = log(Sp);
      const double fv = L.lnNp[sk] + f_old - lnS;
      if (!(Sp >= 1e-290 && Sp <= 1e290)) bad |= FLAG_STATE;
      if (fv != fv) bad |= FLAG_NAN;
      L.fn[sk] = fv;
      if (it == T - 1) {
        if (lnS_out != nullptr) lnS_out[sk] = lnS;
        if (S_out != nullptr) S_out[sk] = Sp;
      }
    }
    __syncthreads();
    // finalisation: gauge, scalars, constants of the next step
    double mdf = 0.0, rs = 0.0, nf = 0.0, gsq = 0.0, minS = INFINITY;
    if (owner) {
      const double fv = L.fn[sk] - L.fn[0];
      f_hist[(int64_t)it * K + sk] = fv;
      double df = fabs(fv - f_old);
      if (df != df) df = INFINITY;
      mdf = df;
      if (sk >= 1) {
        double r;
        if (f_old != 0.0)
          r = fabs(fv / f_old - 1.0);
        else
          r = (fv == 0.0) ? 0.0 : INFINITY;
        if (r != r) r = INFINITY;
        rs = r;
      }
      const double n = L.nk[sk];
      nf = -n * f_old;
      if (n > 0.0) {
        const double g = Sp - n;
        gsq = g * g;
        minS = Sp;
      }
      L.f[sk] = fv;
      L.c[sk] = L.lnNp[sk] + fv;
    }
    if (bad) atomicOr(&L.flags[it & 1], bad);
    // block reduction, waves in order
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      mdf = fmax(mdf, __shfl_xor(mdf, off, 64));
      rs = fmax(rs, __shfl_xor(rs, off, 64));
      nf += __shfl_xor(nf, off, 64);
      gsq += __shfl_xor(gsq, off, 64);
      minS = fmin(minS, __shfl_xor(minS, off, 64));
      obj += __shfl_xor(obj, off, 64);
    }
    if ((tid & 63) == 0) {
      double* r = L.red[tid >> 6];
      r[0] = mdf;
      r[1] = rs;
      r[2] = nf;
      r[3] = gsq;
      r[4] = minS;
      r[5] = obj;
    }
    __syncthreads();
    if (tid == 0) {
      double v[6];
#pragma unroll
      for (int q = 0; q < 6; ++q) v[q] = L.red[0][q];
      for (int w = 1; w < kSB / 64; ++w) {
        v[0] = fmax(v[0], L.red[w][0]);
        v[1] = fmax(v[1], L.red[w][1]);
        v[2] += L.red[w][2];
        v[3] += L.red[w][3];
        v[4] = fmin(v[4], L.red[w][4]);
        v[5] += L.red[w][5];
      }
      SweepScalars o;
      o.max_df = v[0];
      o.rel_step = v[1];
      o.objective = v[5] + v[2];
      o.grad_norm = sqrt(v[3]);
      o.min_S = v[4];
      o.flags = L.flags[it & 1];
      o.pad = 0u;
      scal[it] = o;
    }
  }
  __syncthreads();
  for (int k = tid; k < K; k += kSB) {
    cst[k] = L.c[k];
    gk_out[k] = L.nk[k] > 0.0 ? 1.0 : 0.0;
    lnNp_out[k] = L.lnNp[k];
  }
}

template <int NC>
__device__ __forceinline__ void small_steps(SmallShared<NC>& L, const SmallBatch& a) {
  small_steps<NC>(L, a.u, a.ld, a.K, a.P, a.h, a.Nk, a.f_in, a.T, a.f_hist, a.scal, a.logD,
                  a.lnS, a.S, a.cst, a.gk, a.lnNp);
}

template <int NC>
__global__ void __launch_bounds__(kSB) sci_small_kernel(SmallBatch a) {
  __shared__ SmallShared<NC> L;
  small_steps<NC>(L, a);
}

// The items of column layout NC in a work list (a launch per layout: one
// kernel holding all four bodies would spill registers).
template <int NC>
__global__ void __launch_bounds__(kSB)
    sci_small_fused_kernel(const SmallWorkHeader* __restrict__ wl, int cls) {
  __shared__ SmallShared<NC> L;
  const int64_t count = wl->count[cls];
  const SmallBatch* items = reinterpret_cast<const SmallBatch*>(wl + 1) + wl->first[cls];
  for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
    const SmallBatch a = items[i];
    small_steps<NC>(L, a);
    // the next item reuses the LDS block
    __syncthreads();
  }
}

template <int NC>
constexpr int small_kcap() {
  return (kSB / NC) * kSR;
}

}  // namespace

int small_batch_nc(int K, int64_t P) {
  if (K < 1 || P < 1) return 0;
  if (P <= 64 && K <= small_kcap<64>()) return 64;
  if (P <= 128 && K <= small_kcap<128>()) return 128;
  if (P <= 256 && K <= small_kcap<256>()) return 256;
  if (P <= 512 && K <= small_kcap<512>()) return 512;
  return 0;
}

hipError_t launch_small_batch(hipStream_t s, const SmallBatch& a) {
  const int nc = small_batch_nc(a.K, a.P);
  if (nc == 0 || nc != a.nc || a.T < 1 || a.ld < a.P) return hipErrorInvalidValue;
#define BUMBAR_SMALL(NCV)                                                     \
  if (nc == NCV) {                                                            \
    hipLaunchKernelGGL(sci_small_kernel<NCV>, dim3(1), dim3(kSB), 0, s, a);   \
    return hipGetLastError();                                                 \
  }
  BUMBAR_SMALL(64)
  BUMBAR_SMALL(128)
  BUMBAR_SMALL(256)
  BUMBAR_SMALL(512)
#undef BUMBAR_SMALL
  return hipErrorInvalidValue;
}

int small_class(int nc) {
  return nc == 64 ? 0 : nc == 128 ? 1 : nc == 256 ? 2 : nc == 512 ? 3 : -1;
}

hipError_t launch_small_fused(hipStream_t s, const SmallWorkHeader* wl, unsigned cls_mask,
                              int grid) {
  if (!wl || grid < 1 || grid > kFusedGrid || cls_mask == 0u || cls_mask > 15u)
    return hipErrorInvalidValue;
#define BUMBAR_FUSED(NCV, C)                                                              \
  if (cls_mask & (1u << C)) {                                                             \
    hipLaunchKernelGGL(sci_small_fused_kernel<NCV>, dim3(grid), dim3(kSB), 0, s, wl, C);  \
    const hipError_t e = hipGetLastError();                                               \
    if (e != hipSuccess) return e;                                                        \
  }
  BUMBAR_FUSED(64, 0)
  BUMBAR_FUSED(128, 1)
  BUMBAR_FUSED(256, 2)
  BUMBAR_FUSED(512, 3)
#undef BUMBAR_FUSED
  return hipSuccess;
}

}  // namespace bumbar
