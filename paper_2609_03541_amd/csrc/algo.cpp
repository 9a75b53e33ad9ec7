// Binned stage of BU-MBAR (Algorithm 1, Section 2) on the GPU, plus the
// bumbar_bin entry point.
//
// Readings of the pseudo-code (shared with the CPU oracle): SCI(f, n) is one
// application of Eq. (1) with the binning for target n; in phase 2 the probe
// results are kept (f <- f_next on refinement, otherwise f <- f_new); n is the
// nominal target n0 * inc^t in the Eq. (3) test and in the termination test
// 2 * inc * n > N; comparisons are strict as printed; if the width for
// n * inc equals the width for n (identical binning) the bins are refined at
// once; every binned SCI counts toward max_iter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <utility>

#include "bumbar_impl.h"
#include "solver_internal.h"

namespace bumbar {

constexpr int kCountSlots = 8192;

void BinnedBufs::carve(Arena& ar, int K, int64_t N_, int d_, int num_cus) {
  (void)num_cus;
  d = d_;
  N = N_;
  q = ar.take<uint32_t>((size_t)N * d);
  lo = ar.take<double>(2);
  scale = ar.take<double>(2);
  mm = ar.take<double>(4);
  keys = ar.take<uint64_t>(N);
  keys_sorted = ar.take<uint64_t>(N);
  iota = ar.take<uint32_t>(N);
  perm = ar.take<uint32_t>(N);
  q1_sorted = ar.take<uint32_t>(N);
  perm1 = ar.take<uint32_t>(N);
  bin_of_pos = ar.take<int32_t>(N);
  start = ar.take<int64_t>(N + 1);
  cells = ar.take<uint64_t>(N);
  counts = ar.take<int64_t>(kCountSlots);
  sort_tmp_bytes = sort_temp_bytes(N);
  sort_tmp = ar.take<char>(sort_tmp_bytes);
  for (int i = 0; i < 2; ++i) {
    ubar[i] = ar.take<double>((size_t)K * N);
    h[i] = ar.take<double>(N);
  }
  logD_lvl = ar.take<double>(N);
  f_n = ar.take<double>(K);
  f_x = ar.take<double>(K);
}

void binned_carve_size(Arena& ar, int K, int64_t N, int d, int num_cus) {
  BinnedBufs b;
  b.carve(ar, K, N, d, num_cus);
}

static int quantize_all(bumbar_ctx* ctx, BinnedBufs& BB, const double* xi) {
  hipStream_t s = ctx->stream;
  hipError_t e = launch_minmax(s, xi, BB.N, BB.d, BB.mm, BB.counts);
  if (e == hipSuccess)
    e = launch_quantize(s, xi, BB.N, BB.d, BB.mm, BB.lo, BB.scale, BB.q,
                        reinterpret_cast<unsigned*>(BB.counts + kCountSlots - 1));
  if (e != hipSuccess) return hip_fail(ctx, e, "quantize");
  unsigned bad = 0;
  int rc = read_bytes(ctx, BB.counts + kCountSlots - 1, &bad, sizeof(unsigned));
  if (rc) return rc;
  if (bad) return fail(ctx, BUMBAR_EINVAL, "non-finite binning coordinates");
  if (BB.d == 1) {
    e = launch_sort_1d(s, BB.q, BB.N, BB.iota, BB.q1_sorted, BB.perm1, BB.sort_tmp,
                       BB.sort_tmp_bytes);
    if (e != hipSuccess) return hip_fail(ctx, e, "sort");
  }
  return BUMBAR_OK;
}

static int nonempty(bumbar_ctx* ctx, BinnedBufs& BB, uint64_t m, int64_t* g) {
  hipError_t e;
  if (BB.d == 1)
    e = launch_count_1d(ctx->stream, BB.q1_sorted, BB.N, m, BB.counts);
  else
    e = launch_count_2d(ctx->stream, BB.q, BB.N, m, BB.keys, BB.keys_sorted, BB.sort_tmp,
                        BB.sort_tmp_bytes, BB.counts);
  if (e != hipSuccess) return hip_fail(ctx, e, "count");
  return read_bytes(ctx, BB.counts, g, sizeof(int64_t));
}

// w*(n) = max{m : g(m) >= n} by the integer bisection of the oracle.
static int width_search(bumbar_ctx* ctx, BinnedBufs& BB, int64_t n, uint64_t* m_out,
                        int64_t* g_out) {
  int64_t g1 = 0;
  int rc = nonempty(ctx, BB, 1, &g1);
  if (rc) return rc;
  if (g1 < n) {
    *m_out = 1;
    *g_out = g1;
    return BUMBAR_OK;
  }
  uint64_t lo = 1, hi = 4294967296ull;
  int64_t glo = g1;
  while (hi - lo > 1) {
    const uint64_t mid = lo + (hi - lo) / 2;
    int64_t gm = 0;
    rc = nonempty(ctx, BB, mid, &gm);
    if (rc) return rc;
    if (gm >= n) {
      lo = mid;
      glo = gm;
    } else {
      hi = mid;
    }
  }
  *m_out = lo;
  *g_out = glo;
  return BUMBAR_OK;
}

static int histogram(bumbar_ctx* ctx, BinnedBufs& BB, uint64_t m, int64_t* P) {
  hipError_t e = launch_histogram(ctx->stream, BB.q, BB.N, BB.d, m, BB.q1_sorted, BB.perm1, BB.iota,
                                  BB.keys, BB.keys_sorted, BB.perm, BB.bin_of_pos, BB.start,
                                  BB.cells, BB.sort_tmp, BB.sort_tmp_bytes, BB.counts);
  if (e != hipSuccess) return hip_fail(ctx, e, "histogram");
  return read_bytes(ctx, BB.counts, P, sizeof(int64_t));
}

static int build_level(bumbar_ctx* ctx, BinnedBufs& BB, int K, int64_t n, int model,
                       const double* coef, const double* u, int slot, Level* L) {
  uint64_t m = 0;
  int64_t g = 0;
  int rc = width_search(ctx, BB, n, &m, &g);
  if (rc) return rc;
  int64_t P = 0;
  rc = histogram(ctx, BB, m, &P);
  if (rc) return rc;
  if (P != g) return fail(ctx, BUMBAR_EDEVICE, "histogram size %lld != g(m) %lld", (long long)P,
                          (long long)g);
  hipError_t e = launch_represent(ctx->stream, K, BB.N, BB.d, model, coef, BB.lo, BB.scale, m, P,
                                  BB.cells, BB.start, BB.perm, u, BB.ubar[slot], BB.h[slot]);
  if (e != hipSuccess) return hip_fail(ctx, e, "represent");
  L->n = n;
  L->m = m;
  L->P = P;
  L->ubar = BB.ubar[slot];
  L->h = BB.h[slot];
  return BUMBAR_OK;
}

static int binned_sci(bumbar_ctx* ctx, UnbinnedBufs& B, BinnedBufs& BB, const Level& L,
                      const int64_t* Nk, const double* f, double* f_out, SweepScalars* sc,
                      SweepCounters* cnt) {
  (void)cnt;  // binned sweeps are counted by the stage's iteration counters
  return sweep_at(ctx, B, L.ubar, L.P, L.P, L.h, Nk, f, f_out, BB.logD_lvl, B.lnS_t, B.S_t, sc,
                  false, nullptr);
}

int binned_stage(bumbar_ctx* ctx, UnbinnedBufs& B, BinnedBufs& BB, const double* u,
                 const int64_t* Nk_dev, const int64_t* Nk_host, const double* xi, int d,
                 int model, const double* coef, const bumbar_options& opt, bumbar_stats* st,
                 SweepCounters* cnt) {
  (void)Nk_host;
  hipStream_t s = ctx->stream;
  const int K = B.K;
  const int64_t N = B.N;
  double t_bin = 0.0;
  const double t_start = now_ms();
  double t0 = now_ms();
  int rc = quantize_all(ctx, BB, xi);
  if (rc) return rc;
  (void)d;
  Level cur, nxt;
  int cur_slot = 0;
  int64_t n = opt.n0;
  rc = build_level(ctx, BB, K, n, model, coef, u, cur_slot, &cur);
  if (rc) return rc;
  t_bin += now_ms() - t0;

  // three K-vectors rotate as the current f, SCI(f, n) and SCI(f, n * inc)
  double* slot[3] = {B.f, BB.f_n, BB.f_x};
  int ia = 0;
  SweepScalars sc{};
  int64_t it1 = 0, it2 = 0, nchk = 0;
  int result = BUMBAR_OK;
  // phase 1
  for (;;) {
    if (it1 + it2 >= opt.max_iter) {
      result = BUMBAR_ENOTCONV;
      break;
    }
    const int ib = (ia + 1) % 3;
    rc = binned_sci(ctx, B, BB, cur, Nk_dev, slot[ia], slot[ib], &sc, cnt);
    if (rc) return rc;
    ia = ib;
    ++it1;
    const bool done = opt.replay_refine ? (it1 >= opt.replay_phase1) : (sc.rel_step < opt.eps);
    if (done) break;
  }
  // phase 2
  if (result == BUMBAR_OK) {
    n = n * opt.inc;
    t0 = now_ms();
    rc = build_level(ctx, BB, K, n, model, coef, u, cur_slot, &cur);
    if (rc) return rc;
    rc = build_level(ctx, BB, K, n * opt.inc, model, coef, u, 1 - cur_slot, &nxt);
    if (rc) return rc;
    t_bin += now_ms() - t0;
    for (;;) {
      if (it1 + it2 + opt.n_intermediate + 2 > opt.max_iter) {
        result = BUMBAR_ENOTCONV;
        break;
      }
      for (int i = 0; i < opt.n_intermediate; ++i) {
        const int ib = (ia + 1) % 3;
        rc = binned_sci(ctx, B, BB, cur, Nk_dev, slot[ia], slot[ib], &sc, cnt);
        if (rc) return rc;
        ia = ib;
      }
      const int in = (ia + 1) % 3, ix = (ia + 2) % 3;
      SweepScalars sn{}, sx{};
      rc = binned_sci(ctx, B, BB, cur, Nk_dev, slot[ia], slot[in], &sn, cnt);
      if (rc) return rc;
      rc = binned_sci(ctx, B, BB, nxt, Nk_dev, slot[ia], slot[ix], &sx, cnt);
      if (rc) return rc;
      it2 += opt.n_intermediate + 2;
      int refine;
      if (opt.replay_refine)
        refine = (nchk < opt.n_replay) ? (opt.replay_refine[nchk] != 0) : 0;
      else
        refine = (2.0 * sx.rel_step > (double)opt.inc * sn.rel_step) || (nxt.m == cur.m);
      int stop = 0;
      bumbar_check rec{};
      rec.n = n;
      rec.P = cur.P;
      rec.P_next = nxt.P;
      rec.s_n = sn.rel_step;
      rec.s_next = sx.rel_step;
      rec.refine = refine;
      ia = refine ? ix : in;
      if (refine) {
        n = n * opt.inc;
        if (2 * opt.inc * n > N) stop = 1;
      }
      rec.stop = stop;
      if (st->checks && nchk < st->checks_capacity) st->checks[nchk] = rec;
      ++nchk;
      if (stop) break;
      if (opt.replay_refine && nchk >= opt.n_replay) break;
      if (refine) {
        cur_slot = 1 - cur_slot;
        cur = nxt;
        t0 = now_ms();
        rc = build_level(ctx, BB, K, n * opt.inc, model, coef, u, 1 - cur_slot, &nxt);
        if (rc) return rc;
        t_bin += now_ms() - t0;
      }
    }
  }
  if (slot[ia] != B.f) {
    hipError_t e = hipMemcpyAsync(B.f, slot[ia], sizeof(double) * K, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy f");
  }
  st->phase1_iters = it1;
  st->phase2_iters = it2;
  st->n_checks = nchk;
  st->time_binning_ms = t_bin;
  st->time_binned_ms = now_ms() - t_start - t_bin;
  return result;
}

}  // namespace bumbar

extern "C" int bumbar_bin(bumbar_ctx* ctx, const double* xi, int64_t N, int d, int64_t n_target,
                          void* workspace, size_t ws_bytes, uint64_t* m_out, int64_t* P_out,
                          uint64_t* cells, int64_t* H, int32_t* sample_bin) {
  using namespace bumbar;
  if (!ctx) return BUMBAR_EINVAL;
  ctx->err.clear();
  if (!xi || N <= 0 || d < 1 || d > 2 || n_target < 2 || !workspace || !m_out || !P_out)
    return fail(ctx, BUMBAR_EINVAL, "bad argument");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BUMBAR_EDEVICE, "hipSetDevice");
  Arena ar{reinterpret_cast<char*>(workspace), ws_bytes};
  BinnedBufs BB;
  BB.carve(ar, 1, N, d, ctx->num_cus);
  if (ar.overflow) return fail(ctx, BUMBAR_ENOMEM, "workspace too small");
  int rc = quantize_all(ctx, BB, xi);
  if (rc) return rc;
  uint64_t m = 0;
  int64_t g = 0;
  rc = width_search(ctx, BB, n_target, &m, &g);
  if (rc) return rc;
  int64_t P = 0;
  rc = histogram(ctx, BB, m, &P);
  if (rc) return rc;
  hipStream_t s = ctx->stream;
  hipError_t e = hipSuccess;
  if (cells) e = hipMemcpyAsync(cells, BB.cells, sizeof(uint64_t) * P, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && H) e = launch_counts_from_start(s, P, BB.start, H);
  if (e == hipSuccess && sample_bin) e = launch_sample_bin(s, N, BB.perm, BB.bin_of_pos, sample_bin);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(ctx, e, "bin outputs");
  *m_out = m;
  *P_out = P;
  return BUMBAR_OK;
}
