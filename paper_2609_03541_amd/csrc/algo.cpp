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
#include <functional>
#include <utility>
#include <vector>

#include "bumbar_impl.h"
#include "solver_internal.h"

namespace bumbar {

constexpr int kCountSlots = 8192;
// the 1-D width search keeps its device state at counts + kCountSlots / 2
static_assert(sizeof(WidthSearch1D) <= sizeof(int64_t) * (kCountSlots / 2 - 1),
              "width-search state must fit below the last count slot");
static_assert(sizeof(WidthSearch2D) <= sizeof(int64_t) * (kCountSlots / 2 - 1),
              "width-search state must fit below the last count slot");

// Bins per level whose centre representatives are materialised (K <= 256):
// at least 65536, and N / 8, which covers the levels of nominal size up to
// N / 10 that Algorithm 1 reaches before it stops refining; larger levels run
// the model sweep at their centres. Two level slots of K x cap doubles then
// cost 2 K N bytes at most beyond 65536 bins, not 16 K N.
int64_t otf_ubar_cap(int K, int64_t N) {
  return sweep_fast_supported(K) || sweep_smaj_supported(K)
             ? std::min<int64_t>(N, std::max<int64_t>(65536, N / 8))
             : 0;
}

// Values per bin of a materialised level: K (state-major, K <= 256) or the
// sample-major row Kp (256 < K <= 1024).
static int level_row(int K) { return sweep_fast_supported(K) ? K : smaj_row(K); }

void BinnedBufs::carve(Arena& ar, int K, int64_t N_, int d_, int num_cus, bool ubar_bufs,
                       bool cen_bufs, bool cen_f32, int64_t otf_cap) {
  otf = cen_bufs && !ubar_bufs;
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
  if (d == 1) {
    q1_sorted = ar.take<uint32_t>(N);
    perm1 = ar.take<uint32_t>(N);
  } else {
    q2_sorted = ar.take<uint64_t>(N);
  }
  bin_of_pos = ar.take<int32_t>(N);
  start = ar.take<int64_t>(N + 1);
  cells = ar.take<uint64_t>(N);
  counts = ar.take<int64_t>(kCountSlots);
  sort_tmp_bytes = sort_temp_bytes(N);
  sort_tmp = ar.take<char>(sort_tmp_bytes);
  for (int i = 0; i < 2; ++i) {
    if (cen_bufs) cen[i] = ar.take<double>((size_t)N * d);
    if (cen_bufs && cen_f32) cenf[i] = ar.take<float>((size_t)N * d);
    if (ubar_bufs)
      ubar[i] = ar.take<double>((size_t)K * N);
    else if (otf_cap > 0)
      ubar[i] = ar.take<double>((size_t)level_row(K) * otf_cap);
    h[i] = ar.take<double>(N);
  }
  ubar_cap = ubar_bufs ? N : otf_cap;
  ubar_row = ubar_bufs ? K : level_row(K);
  logD_lvl = ar.take<double>(N);
  if (smaj_batch_supported(K)) coop = ar.take<double>(smaj_batch_scratch(num_cus, kHistSteps));
  f_n = ar.take<double>(K);
  f_x = ar.take<double>(K);
}

void binned_carve_size(Arena& ar, int K, int64_t N, int d, int num_cus, bool ubar_bufs,
                       bool cen_bufs, bool cen_f32, int64_t otf_cap) {
  BinnedBufs b;
  b.carve(ar, K, N, d, num_cus, ubar_bufs, cen_bufs, cen_f32, otf_cap);
}

static int quantize_all(bumbar_ctx* ctx, BinnedBufs& BB, const double* xi) {
  hipStream_t s = ctx->stream;
  BB.g1 = -1;  // recounted for the new quantisation
  hipError_t e = launch_minmax(s, xi, BB.N, BB.d, BB.mm, BB.counts);
  if (e == hipSuccess)
    e = launch_quantize(s, xi, BB.N, BB.d, BB.mm, BB.lo, BB.scale, BB.q,
                        reinterpret_cast<unsigned*>(BB.counts + kCountSlots - 1));
  if (e != hipSuccess) return hip_fail(ctx, e, "quantize");
  unsigned bad = 0;
  int rc = read_bytes(ctx, BB.counts + kCountSlots - 1, &bad, sizeof(unsigned));
  if (rc) return rc;
  if (bad) return fail(ctx, BUMBAR_EINVAL, "non-finite binning coordinates");
  if (BB.d == 1)
    e = launch_sort_1d(s, BB.q, BB.N, BB.iota, BB.q1_sorted, BB.perm1, BB.sort_tmp,
                       BB.sort_tmp_bytes);
  else
    e = launch_sort_2d(s, BB.q, BB.N, BB.keys, BB.q2_sorted, BB.sort_tmp, BB.sort_tmp_bytes);
  if (e != hipSuccess) return hip_fail(ctx, e, "sort");
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

// 1-D: the same bisection, run on the device: each pass counts the midpoints
// of the next k levels of the bisection tree over the sorted coordinates, and
// a one-thread kernel walks the path exactly as the bisection would and
// queues the next pass, so the passes run back to back and the host reads
// back only the result. A pass costs a few microseconds of launches plus
// N x 2^k lane steps of the count kernel (about 0.32 ps each on MI355X); k
// minimises ceil(32 / k) passes of that: 4 levels at N = 1e6, 2 at 1e7.
static int bisection_levels(int64_t N) {
  int best = 6;
  double best_us = 1e300;
  for (int k = 1; k <= 6; ++k) {
    const double us = std::ceil(32.0 / k) * (6.0 + (double)N * (double)(1 << k) * 3.2e-7);
    if (us < best_us) {
      best_us = us;
      best = k;
    }
  }
  return best;
}

static int width_search_1d(bumbar_ctx* ctx, BinnedBufs& BB, int64_t n, uint64_t* m_out,
                           int64_t* g_out) {
  hipStream_t s = ctx->stream;
  auto* w = reinterpret_cast<WidthSearch1D*>(BB.counts + kCountSlots / 2);
  const int levels = bisection_levels(BB.N);
  // 32 levels cover [1, 2^32]; one spare pass
  int passes = (32 + levels - 1) / levels + 1;
  bool init = true;
  WidthSearch1D h;
  for (int round = 0; round < 4; ++round) {
    hipError_t e = launch_width_search_1d(s, BB.q1_sorted, BB.N, n, levels, passes, init, w);
    if (e != hipSuccess) return hip_fail(ctx, e, "width search");
    const int rc = read_bytes(ctx, w, &h, sizeof(h));
    if (rc) return rc;
    if (h.done) {
      *m_out = h.lo;
      *g_out = h.glo;
      return BUMBAR_OK;
    }
    init = false;
    passes = 4;
  }
  return fail(ctx, BUMBAR_EDEVICE, "the width search did not end");
}

// w*(n) = max{m : g(m) >= n} by the integer bisection of the oracle.
static int width_search(bumbar_ctx* ctx, BinnedBufs& BB, int64_t n, uint64_t* m_out,
                        int64_t* g_out) {
  if (BB.d == 1) return width_search_1d(ctx, BB, n, m_out, g_out);
  // g(1): the runs of the sorted pairs; the coordinates do not change within
  // a solve
  int rc = BUMBAR_OK;
  if (BB.g1 < 0) {
    const hipError_t e = launch_count_sorted_2d(ctx->stream, BB.q2_sorted, BB.N, BB.counts);
    if (e != hipSuccess) return hip_fail(ctx, e, "count");
    rc = read_bytes(ctx, BB.counts, &BB.g1, sizeof(int64_t));
    if (rc) return rc;
  }
  const int64_t g1 = BB.g1;
  if (g1 < n) {
    *m_out = 1;
    *g_out = g1;
    return BUMBAR_OK;
  }
  uint64_t lo = 1, hi = 4294967296ull;
  int64_t glo = g1;
  // the probes whose grids fit the bitmap run on the device, queued back to
  // back (32 bisection steps at most); the host takes over where a grid does
  // not fit, from the same (lo, hi, g(lo))
  {
    auto* w = reinterpret_cast<WidthSearch2D*>(BB.counts + kCountSlots / 2);
    hipError_t e =
        launch_width_search_2d(ctx->stream, BB.q2_sorted, BB.N, n, g1, 33, true, BB.keys, w);
    if (e != hipSuccess) return hip_fail(ctx, e, "width search");
    WidthSearch2D h;
    rc = read_bytes(ctx, w, &h, sizeof(h));
    if (rc) return rc;
    lo = h.lo;
    hi = h.hi;
    glo = h.glo;
    if (h.done || hi - lo <= 1) {
      *m_out = lo;
      *g_out = glo;
      return BUMBAR_OK;
    }
  }
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

// Batches of binned SCI steps as HIP graphs. A batch (the steps queued
// between two readbacks) is fixed by its kind, its length and the levels it
// runs on, since all of its buffers are the stage's own; the first batch of
// each shape is captured on the context's capture stream (nothing runs
// there) and that batch and every later one of the shape launch the graph on
// the working stream. A batch is 40 to 150 kernel launches, so this replaces
// as many host launches by one. The graphs hold kernel launches only. If
// capture or instantiation fails, the batch and the rest of the stage are
// launched kernel by kernel.
struct BatchKey {
  int kind;
  int64_t T;
  const void* a;
  int64_t pa;
  const void* b;
  int64_t pb;
  bool operator==(const BatchKey& o) const {
    return kind == o.kind && T == o.T && a == o.a && pa == o.pa && b == o.b && pb == o.pb;
  }
};

class BatchGraphs {
 public:
  BatchGraphs(bumbar_ctx* ctx, bool on) : ctx_(ctx), on_(on) {}
  ~BatchGraphs() {
    for (auto& x : execs_) (void)hipGraphExecDestroy(x.second);
  }
  BatchGraphs(const BatchGraphs&) = delete;
  BatchGraphs& operator=(const BatchGraphs&) = delete;

  // enqueue(): queues the batch on ctx->stream, returns a BUMBAR_* code
  template <class F>
  int run(const BatchKey& k, F&& enqueue) {
    if (!on_) return enqueue();
    for (auto& x : execs_)
      if (x.first == k) return launch(x.second);
    if (!ctx_->cap_stream &&
        hipStreamCreateWithFlags(&ctx_->cap_stream, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      ctx_->cap_stream = nullptr;
      on_ = false;
      return enqueue();
    }
    if (hipStreamBeginCapture(ctx_->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
      (void)hipGetLastError();
      on_ = false;
      return enqueue();
    }
    hipStream_t work = ctx_->stream;
    ctx_->stream = ctx_->cap_stream;
    const int rc = enqueue();
    ctx_->stream = work;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx_->cap_stream, &g);
    // a batch whose work went to another stream captures nothing, and its
    // replays would do nothing: refuse it
    size_t nodes = 0;
    if (rc == BUMBAR_OK && e == hipSuccess && hipGraphGetNodes(g, nullptr, &nodes) == hipSuccess &&
        nodes == 0) {
      (void)hipGraphDestroy(g);
      return fail(ctx_, BUMBAR_EDEVICE, "a captured batch of binned steps holds no work");
    }
    hipGraphExec_t x = nullptr;
    if (rc == BUMBAR_OK && e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (rc != BUMBAR_OK) return rc;
    if (e != hipSuccess) {
      (void)hipGetLastError();
      on_ = false;
      return enqueue();
    }
    execs_.emplace_back(k, x);
    return launch(x);
  }
  int64_t launched() const { return launched_; }

 private:
  int launch(hipGraphExec_t x) {
    const hipError_t e = hipGraphLaunch(x, ctx_->stream);
    if (e != hipSuccess) return hip_fail(ctx_, e, "graph launch");
    ++launched_;
    return BUMBAR_OK;
  }
  bumbar_ctx* ctx_;
  bool on_;
  int64_t launched_ = 0;
  std::vector<std::pair<BatchKey, hipGraphExec_t>> execs_;
};

// Identity of a level's matrix for BatchKey: its representatives or centres
// (the buffers of its slot) and its bin count.
static const void* level_id(const Level& L) {
  return L.ubar ? static_cast<const void*>(L.ubar) : static_cast<const void*>(L.cen);
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
  hipError_t e;
  if (BB.otf)
    e = launch_centres(ctx->stream, BB.d, BB.lo, BB.scale, m, P, BB.cells, BB.start,
                       BB.cen[slot], BB.h[slot]);
  else
    e = launch_represent(ctx->stream, K, BB.N, BB.d, model, coef, BB.lo, BB.scale, m, P,
                         BB.cells, BB.start, BB.perm, u, BB.ubar[slot], BB.h[slot]);
  if (e == hipSuccess && BB.otf && BB.cenf[slot])
    e = launch_pack_coords(ctx->stream, P * BB.d, BB.cen[slot], BB.cenf[slot]);
  // a level of at most ubar_cap bins with bin-centre representatives: the
  // representatives once (state-major for K <= 256, sample-major above), then
  // the steps of the level are one-pass sweeps over them
  const bool mat = BB.otf && BB.ubar[slot] && P <= BB.ubar_cap;
  const bool smaj = mat && BB.ubar_row != K;
  if (e == hipSuccess && mat && !smaj)
    e = launch_represent(ctx->stream, K, BB.N, BB.d, model, coef, BB.lo, BB.scale, m, P, BB.cells,
                         BB.start, BB.perm, nullptr, BB.ubar[slot], BB.h[slot]);
  if (e == hipSuccess && smaj)
    e = launch_represent_smaj(ctx->stream, K, BB.ubar_row, BB.d, model, coef, P, BB.cen[slot],
                              BB.ubar[slot]);
  if (e != hipSuccess) return hip_fail(ctx, e, "represent");
  L->n = n;
  L->m = m;
  L->P = P;
  L->smaj = smaj;
  L->ubar = (!BB.otf || mat) ? BB.ubar[slot] : nullptr;
  L->cen = BB.otf ? BB.cen[slot] : nullptr;
  L->cenf = BB.otf ? BB.cenf[slot] : nullptr;
  L->h = BB.h[slot];
  return BUMBAR_OK;
}

// The matrix of a level: stored representatives, or the model evaluated at
// the bin centres when the stage runs on the fly (FP32 when the level has
// FP32 centres and fp32 is asked for, else FP64).
static Mat level_mat_of(const Level& L, const Mat* otf_base, bool fp32) {
  // a small on-the-fly level has its representatives materialised (used
  // unless FP32 centre steps are asked for)
  const bool stored = L.ubar != nullptr && !(fp32 && L.cenf);
  if (otf_base && !stored) {
    Mat M = *otf_base;
    M.kind = (fp32 && L.cenf) ? 3 : 4;
    M.otf.xi = L.cen;
    M.otf.xf = L.cenf;
    return M;
  }
  Mat M;
  M.u = L.ubar;
  M.kind = 0;
  M.ld = L.P;
  if (L.smaj) {
    // the sample-major sweep over the level's rows (finite model values)
    M.ut = L.ubar;
    M.ut_f32 = false;
    M.ut_checked = true;
  }
  return M;
}

int binned_stage(bumbar_ctx* ctx, UnbinnedBufs& B, BinnedBufs& BB, const double* u,
                 const int64_t* Nk_dev, const int64_t* Nk_host, const double* xi, int d,
                 int model, const double* coef, const bumbar_options& opt, bumbar_stats* st,
                 SweepCounters* cnt, const Mat* otf_base, bool fp32_steps) {
  // batched steps: FP32 centres when asked for (and present); the
  // one-at-a-time fallback steps: FP64
  auto level_mat = [otf_base, fp32_steps](const Level& L) {
    return level_mat_of(L, otf_base, fp32_steps);
  };
  auto level_mat64 = [otf_base](const Level& L) { return level_mat_of(L, otf_base, false); };
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

  // The current f lives in BB.f_n. Steps are queued in batches whose iterates
  // go to B.f_hist and whose scalars go to B.scal_hist; one readback per
  // batch. The decisions use exactly the per-step values, so the trajectory
  // is the same as with a readback after every step; a flagged step (far-off
  // f, see the sweep) is redone on the robust path before anything else.
  hipError_t e = hipMemcpyAsync(BB.f_n, B.f, sizeof(double) * K, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "copy f");
  // batched steps need a kernel that flags the rare steps that need the
  // robust rerun: the register-tiled FP64 sweep, or the model sweep
  const bool fast = otf_base != nullptr || sweep_fast_supported(K);
  std::vector<SweepScalars> hs(kHistSteps);
  auto fh = [&](int i) { return B.f_hist + (size_t)i * K; };
  auto set_current = [&](const double* src) -> int {
    hipError_t e2 = hipMemcpyAsync(BB.f_n, src, sizeof(double) * K, hipMemcpyDeviceToDevice, s);
    return e2 == hipSuccess ? BUMBAR_OK : hip_fail(ctx, e2, "copy f");
  };
  auto read_hist = [&](int T) -> int {
    return read_bytes(ctx, B.scal_hist, hs.data(), sizeof(SweepScalars) * T);
  };
  auto flagged = [&](const SweepScalars& x) {
    return (x.flags & (FLAG_COL | FLAG_STATE | FLAG_NAN)) != 0;
  };
  // one step on the robust-capable path, result in fh(slot)
  auto safe_step = [&](const Level& L, const double* fin, int slot, SweepScalars* sc) -> int {
    return sweep_at(ctx, B, level_mat64(L), L.P, L.h, Nk_dev, fin, fh(slot), BB.logD_lvl,
                    B.lnS_t, B.S_t, sc, false, nullptr);
  };
  // a batch of steps on a stored level of at most 512 bins: one workgroup
  // with the matrix in registers runs them all (same outputs per step);
  // counted after each batch, since a graph replay does not call the lambda
  int64_t batched = 0, coop_steps = 0;
  auto small_level = [&](const Level& L) {
    const Mat M = level_mat(L);
    return M.kind == 0 && M.u != nullptr && M.ut == nullptr && small_batch_nc(K, L.P) != 0;
  };
  // a batch of steps on a level materialised sample-major (256 < K <= 1024):
  // one cooperative launch (same outputs per step as sweep and finaliser)
  auto coop_level = [&](const Level& L) {
    if (!opt.grid_batches || !ctx->coop_ok || BB.coop == nullptr) return false;
    const Mat M = level_mat(L);
    return M.kind == 0 && M.ut != nullptr && !M.ut_f32 && smaj_batch_supported(K);
  };
  auto coop_batch = [&](const Level& L, const double* fin, int T) -> int {
    const Mat M = level_mat(L);
    hipError_t e2 = launch_smaj_batch(ctx->stream, static_cast<const double*>(M.ut), K, L.P, L.h,
                                      Nk_dev, fin, T, fh(0), B.scal_hist, BB.logD_lvl, B.lnS_t,
                                      B.S_t, B.cst, B.gk, B.lnNp, B.part, B.nparts_cap, BB.coop,
                                      kHistSteps, ctx->num_cus);
    if (e2 != hipSuccess) {
      // no co-resident grid for it on this device: the per-step kernels from now on
      (void)hipGetLastError();
      ctx->coop_ok = false;
      return -1;
    }
    coop_steps += T;
    return BUMBAR_OK;
  };
  auto small_batch = [&](const Level& L, const double* fin, int T) -> int {
    const Mat M = level_mat(L);
    SmallBatch a;
    a.u = reinterpret_cast<const double*>(M.u);
    a.ld = M.ld;
    a.h = L.h;
    a.Nk = Nk_dev;
    a.f_in = fin;
    a.f_hist = fh(0);
    a.scal = B.scal_hist;
    a.logD = BB.logD_lvl;
    a.lnS = B.lnS_t;
    a.S = B.S_t;
    a.cst = B.cst;
    a.gk = B.gk;
    a.lnNp = B.lnNp;
    a.K = K;
    a.P = (int)L.P;
    a.T = T;
    a.nc = small_batch_nc(K, L.P);
    // a fusing server takes the batch into its next fused launch
    if (ctx->post_small) return ctx->post_small(ctx->post_arg, a);
    // ctx->stream, not s: while a batch is captured it names the capture stream
    hipError_t e2 = launch_small_batch(ctx->stream, a);
    return e2 == hipSuccess ? BUMBAR_OK : hip_fail(ctx, e2, "small batch");
  };

  int64_t it1 = 0, it2 = 0, nchk = 0;
  int result = BUMBAR_OK;
  BatchGraphs graphs(ctx, opt.graphs != 0);
  // batches handed to a fusing server are not captured here (the server
  // launches them), nor are cooperative batches; every other batch goes
  // through the graphs
  auto run_batch = [&](const BatchKey& key, const Level& L, bool small_part,
                       const std::function<int()>& enqueue) -> int {
    if (small_part && ((ctx->post_small && small_level(L)) || coop_level(L))) return enqueue();
    return graphs.run(key, enqueue);
  };  // ---- phase 1: iterate at n0 until the relative step is below eps ----
  for (bool done = false; !done;) {
    if (it1 + it2 >= opt.max_iter) {
      result = BUMBAR_ENOTCONV;
      break;
    }
    int64_t T = std::min<int64_t>(kHistSteps, opt.max_iter - it1 - it2);
    if (opt.replay_refine) T = std::min<int64_t>(T, std::max<int64_t>(1, opt.replay_phase1 - it1));
    int nvalid = 0;  // leading steps that are usable
    if (fast) {
      rc = run_batch({1, T, level_id(cur), cur.P, nullptr, 0}, cur, true, [&]() -> int {
        if (small_level(cur)) return small_batch(cur, BB.f_n, (int)T);
        if (coop_level(cur)) {
          const int r = coop_batch(cur, BB.f_n, (int)T);
          if (r != -1) return r;
        }
        for (int i = 0; i < T; ++i) {
          // each step's finaliser leaves the constants of the next step in B.cst
          const int r = sweep_queue(ctx, B, level_mat(cur), cur.P, cur.h, Nk_dev,
                                    i == 0 ? BB.f_n : fh(i - 1), fh(i), BB.logD_lvl, B.lnS_t,
                                    B.S_t, B.scal_hist + i, i > 0, B.cst);
          if (r) return r;
        }
        return BUMBAR_OK;
      });
      if (rc) return rc;
      if (small_level(cur)) batched += T;
      rc = read_hist((int)T);
      if (rc) return rc;
      while (nvalid < T && !flagged(hs[nvalid])) ++nvalid;
    }
    if (nvalid == 0) {  // first step flagged (or no fast path): one robust-capable step
      rc = safe_step(cur, BB.f_n, 0, &hs[0]);
      if (rc) return rc;
      nvalid = 1;
    }
    int used = nvalid;
    for (int i = 0; i < nvalid; ++i) {
      const int64_t n_it = it1 + i + 1;
      const bool stop = opt.replay_refine ? (n_it >= opt.replay_phase1) : (hs[i].rel_step < opt.eps);
      if (stop) {
        used = i + 1;
        done = true;
        break;
      }
    }
    it1 += used;
    rc = set_current(fh(used - 1));
    if (rc) return rc;
  }
  // ---- phase 2 ----
  if (result == BUMBAR_OK) {
    n = n * opt.inc;
    t0 = now_ms();
    rc = build_level(ctx, BB, K, n, model, coef, u, cur_slot, &cur);
    if (rc) return rc;
    rc = build_level(ctx, BB, K, n * opt.inc, model, coef, u, 1 - cur_slot, &nxt);
    if (rc) return rc;
    t_bin += now_ms() - t0;
    const int nint = opt.n_intermediate;
    for (;;) {
      if (it1 + it2 + nint + 2 > opt.max_iter) {
        result = BUMBAR_ENOTCONV;
        break;
      }
      // intermediate steps, in batches that leave room for the two probes
      int done_int = 0;
      bool fallback = false;
      while (!fallback && nint - done_int > kHistSteps - 2) {
        const int T = kHistSteps - 2;
        if (!fast) {
          fallback = true;
          break;
        }
        rc = run_batch({2, T, level_id(cur), cur.P, nullptr, 0}, cur, true, [&]() -> int {
          if (small_level(cur)) return small_batch(cur, BB.f_n, T);
          if (coop_level(cur)) {
            const int r = coop_batch(cur, BB.f_n, T);
            if (r != -1) return r;
          }
          for (int i = 0; i < T; ++i) {
            const int r = sweep_queue(ctx, B, level_mat(cur), cur.P, cur.h, Nk_dev,
                                      i == 0 ? BB.f_n : fh(i - 1), fh(i), BB.logD_lvl, B.lnS_t,
                                      B.S_t, B.scal_hist + i, i > 0, B.cst);
            if (r) return r;
          }
          return BUMBAR_OK;
        });
        if (rc) return rc;
        if (small_level(cur)) batched += T;
        rc = read_hist(T);
        if (rc) return rc;
        for (int i = 0; i < T; ++i) fallback = fallback || flagged(hs[i]);
        if (fallback) break;
        rc = set_current(fh(T - 1));
        if (rc) return rc;
        done_int += T;
      }
      SweepScalars sn{}, sx{};
      int in = 0, ix = 0;
      if (!fallback && fast) {
        const int T = nint - done_int;
        in = T;
        ix = T + 1;
        rc = run_batch({3, T, level_id(cur), cur.P, level_id(nxt), nxt.P}, cur, T > 0,
                       [&]() -> int {
          int rc_coop = -1;
          if (T > 0 && !small_level(cur) && coop_level(cur)) rc_coop = coop_batch(cur, BB.f_n, T);
          if (rc_coop != -1 && rc_coop != BUMBAR_OK) return rc_coop;
          if (T > 0 && small_level(cur)) {
            const int r = small_batch(cur, BB.f_n, T);
            if (r) return r;
          } else if (rc_coop != BUMBAR_OK) {
            for (int i = 0; i < T; ++i) {
              const int r = sweep_queue(ctx, B, level_mat(cur), cur.P, cur.h, Nk_dev,
                                        i == 0 ? BB.f_n : fh(i - 1), fh(i), BB.logD_lvl,
                                        B.lnS_t, B.S_t, B.scal_hist + i, i > 0, B.cst);
              if (r) return r;
            }
          }
          const double* fin = T == 0 ? BB.f_n : fh(T - 1);
          // both probes start from fin: the first reuses the constants the last
          // intermediate step left (if any), the second those of the first
          int r = sweep_queue(ctx, B, level_mat(cur), cur.P, cur.h, Nk_dev, fin, fh(in),
                              BB.logD_lvl, B.lnS_t, B.S_t, B.scal_hist + in, T > 0, nullptr);
          if (r) return r;
          r = sweep_queue(ctx, B, level_mat(nxt), nxt.P, nxt.h, Nk_dev, fin, fh(ix), BB.logD_lvl,
                          B.lnS_t, B.S_t, B.scal_hist + ix, true, nullptr);
          return r;
        });
        if (rc) return rc;
        if (T > 0 && small_level(cur)) batched += T;
        rc = read_hist(T + 2);
        if (rc) return rc;
        for (int i = 0; i < T + 2; ++i) fallback = fallback || flagged(hs[i]);
        sn = hs[in];
        sx = hs[ix];
      }
      if (fallback || !fast) {
        // redo the remaining intermediate steps and both probes one by one from
        // the current f (robust path where a step needs it)
        for (int i = done_int; i < nint; ++i) {
          rc = safe_step(cur, BB.f_n, 0, nullptr);
          if (rc) return rc;
          rc = set_current(fh(0));
          if (rc) return rc;
        }
        in = 0;
        ix = 1;
        rc = safe_step(cur, BB.f_n, in, &sn);
        if (rc) return rc;
        rc = safe_step(nxt, BB.f_n, ix, &sx);
        if (rc) return rc;
      }
      it2 += nint + 2;
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
      rc = set_current(refine ? fh(ix) : fh(in));
      if (rc) return rc;
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
  e = hipMemcpyAsync(B.f, BB.f_n, sizeof(double) * K, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "copy f");
  st->phase1_iters = it1;
  st->phase2_iters = it2;
  st->n_checks = nchk;
  st->graph_batches += graphs.launched();
  st->batched_steps += batched;
  st->coop_steps += coop_steps;
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
  BB.carve(ar, 1, N, d, ctx->num_cus, false, false);
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
