// Host side of libbumbar: the C ABI of include/bumbar.h, the unbinned sweep
// driver (fast path with robust fallback) and the Newton finisher.
//
// The binned stage (Algorithm 1) lives in algo.cpp; both use the helpers
// declared in solver_internal.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <vector>

#include "bumbar_impl.h"
#include "solver_internal.h"

using namespace bumbar;

namespace bumbar {

int fail(bumbar_ctx* ctx, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  return code;
}

int hip_fail(bumbar_ctx* ctx, hipError_t e, const char* where) {
  return fail(ctx, BUMBAR_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Device buffers of one unbinned problem, carved from the workspace.
void UnbinnedBufs::carve(Arena& ar, int K_, int64_t N_, int num_cus) {
  K = K_;
  N = N_;
  cst = ar.take<double>(K);
  gk = ar.take<double>(K);
  lnNp = ar.take<double>(K);
  f = ar.take<double>(K);
  f_new = ar.take<double>(K);
  f_trial = ar.take<double>(K);
  dir = ar.take<double>(K);
  f_sweep = ar.take<double>(K);
  lnS = ar.take<double>(K);
  S = ar.take<double>(K);
  lnS_t = ar.take<double>(K);
  S_t = ar.take<double>(K);
  logD = ar.take<double>(N);
  logD_t = ar.take<double>(N);
  const int g = sweep_max_grid(num_cus);
  const int ch = robust_chunks(N);
  nparts_cap = std::max(g, ch);
  part = ar.take<double>((size_t)nparts_cap * K);
  partS = ar.take<double>((size_t)ch * K);
  part_obj = ar.take<double>(nparts_cap);
  part_flags = ar.take<unsigned>(nparts_cap);
  scal = ar.take<SweepScalars>(2);
  scal_hist = ar.take<SweepScalars>(kHistSteps);
  f_hist = ar.take<double>((size_t)kHistSteps * K);
  misc = ar.take<double>(8);
  ok = ar.take<int>(4);
  nan_flag = ar.take<unsigned>(1);
  idx = ar.take<int>(K);
  A = ar.take<double>(newton_ws_doubles(K));
  H = ar.take<double>((size_t)K * K);
  hess_parts = ar.take<double>(hessian_partial_count(K, N, num_cus, &hess_chunks));
  dk = ar.take<double>(K);
}

// Event pairs for timing sweep kernels; at most 4096 launches per solve are timed.
std::pair<hipEvent_t, hipEvent_t>* next_event_pair(bumbar_ctx* ctx) {
  if (ctx->events_used >= 4096) return nullptr;
  if (ctx->events_used == ctx->events.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return nullptr;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return nullptr;
    }
    ctx->events.emplace_back(a, b);
  }
  return &ctx->events[ctx->events_used++];
}

// Sum of the timed intervals (the stream must have been synchronised).
static double collect_event_ms(bumbar_ctx* ctx, int64_t* count) {
  double tot = 0.0;
  for (size_t i = 0; i < ctx->events_used; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->events[i].first, ctx->events[i].second) == hipSuccess)
      tot += ms;
  }
  *count = (int64_t)ctx->events_used;
  ctx->events_used = 0;
  return tot;
}

hipError_t ctx_wait(bumbar_ctx* ctx, hipStream_t s) {
  if (!ctx->yield) return hipStreamSynchronize(s);
  for (;;) {
    const hipError_t q = hipStreamQuery(s);
    if (q != hipErrorNotReady) return q;
    ctx->yield(ctx->yield_arg);
  }
}

int read_scalars(bumbar_ctx* ctx, const SweepScalars* dev, SweepScalars* host) {
  hipError_t e = hipMemcpyAsync(ctx->pinned, dev, sizeof(SweepScalars), hipMemcpyDeviceToHost,
                                ctx->stream);
  if (e == hipSuccess) e = ctx_wait(ctx, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "scalar readback");
  std::memcpy(host, ctx->pinned, sizeof(SweepScalars));
  return BUMBAR_OK;
}

int read_bytes(bumbar_ctx* ctx, const void* dev, void* host, size_t bytes) {
  // small readbacks go through the context's pinned buffer: an asynchronous
  // DMA, with no staging through the runtime's shared pageable-copy buffers
  // (which serialise the readbacks of concurrent solves)
  if (bytes <= kPinnedBytes) {
    hipError_t e = hipMemcpyAsync(ctx->pinned, dev, bytes, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = ctx_wait(ctx, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "readback");
    std::memcpy(host, ctx->pinned, bytes);
    return BUMBAR_OK;
  }
  // a copy into pageable memory blocks the host until the stream reaches it:
  // a fiber first lets the stream drain
  hipError_t e = ctx->yield ? ctx_wait(ctx, ctx->stream) : hipSuccess;
  if (e == hipSuccess) e = hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = ctx_wait(ctx, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "readback");
  return BUMBAR_OK;
}

// One sweep (unbinned when h == nullptr, binned with multiplicities h
// otherwise) of the matrix M at f. Outputs: f_out (gauged SCI step),
// logD_out, lnS_out, S_out and the scalars (read back to *sc when sc != null).
// Kernel choice: FP64 u with K <= 256 -> register-tiled single pass; other
// FP64 / FP32 u -> two-pass FP64; packed matrix -> FP32 single pass; model
// kinds -> on-the-fly passes. A flagged FP64 sweep is redone on the robust
// path.
static int queue_sweep(bumbar_ctx* ctx, const UnbinnedBufs& B, const Mat& M, int64_t N,
                       const double* h, const int64_t* Nk, const double* f, double* f_out,
                       double* logD_out, double* lnS_out, double* S_out, SweepScalars* dev_scal,
                       bool timed, bool consts_ready = false, double* cst_next = nullptr) {
  hipStream_t s = ctx->stream;
  const int K = B.K;
  hipError_t e = hipSuccess;
  if (!consts_ready) e = launch_prepare_consts(s, K, Nk, f, B.cst, B.gk, B.lnNp);
  if (e != hipSuccess) return hip_fail(ctx, e, "prepare_consts");
  int grid = 0;
  std::pair<hipEvent_t, hipEvent_t>* ev = nullptr;
  if (timed && ctx->profiling && h == nullptr) ev = next_event_pair(ctx);
  if (M.ut != nullptr) {
    // the sample-major copy (FP64 arithmetic, or FP32 for kind 7)
    if (ev) (void)hipEventRecord(ev->first, s);
    e = launch_sweep_smaj(s, M.ut, M.ut_f32, M.kind == 7, !M.ut_checked, K, N, B.cst, B.gk, h,
                          logD_out, B.part, B.part_obj, B.part_flags, ctx->num_cus, &grid);
  } else if (M.kind == 2) {
    e = launch_delta(s, K, f, M.f0, B.dk);
    if (e != hipSuccess) return hip_fail(ctx, e, "delta");
    if (ev) (void)hipEventRecord(ev->first, s);
    e = launch_sweep32(s, reinterpret_cast<const float*>(M.u), M.ld, K, N, B.dk, B.gk, M.m0,
                       logD_out, B.part, B.part_obj, B.part_flags, ctx->num_cus, &grid);
  } else if (M.kind == 7) {
    // FP32 exponentials over the stored FP32 u (K <= 256), no copy
    if (ev) (void)hipEventRecord(ev->first, s);
    e = launch_sweep_fast(s, M.u, true, true, M.ld, K, N, B.cst, B.gk, h, logD_out, B.part,
                          B.part_obj, B.part_flags, ctx->num_cus, &grid);
  } else if (M.kind >= 3) {
    if (ev) (void)hipEventRecord(ev->first, s);
    e = launch_sweep_otf(s, M.otf, M.kind == 3, K, N, B.cst, B.gk, h, logD_out, B.part,
                         (size_t)B.nparts_cap * K, B.part_obj, B.part_flags, ctx->num_cus, &grid);
  } else if ((M.kind == 0 || M.kind == 1) && sweep_fast_supported(K)) {
    if (ev) (void)hipEventRecord(ev->first, s);
    e = launch_sweep_fast(s, M.u, M.kind == 1, false, M.ld, K, N, B.cst, B.gk, h, logD_out,
                          B.part, B.part_obj, B.part_flags, ctx->num_cus, &grid);
  } else {
    if (ev) (void)hipEventRecord(ev->first, s);
    e = launch_sweep_wide(s, M.u, M.kind == 1, M.ld, K, N, B.cst, B.gk, h, logD_out, B.part,
                          B.part_obj, B.part_flags, ctx->num_cus, &grid);
  }
  if (ev) (void)hipEventRecord(ev->second, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "sweep");
  e = launch_sweep_finalize(s, 0, K, grid, B.part, B.partS, B.part_obj, B.part_flags, f, B.lnNp,
                            Nk, f_out, lnS_out, S_out, dev_scal, cst_next);
  if (e != hipSuccess) return hip_fail(ctx, e, "sweep_finalize");
  return BUMBAR_OK;
}

int sweep_queue(bumbar_ctx* ctx, const UnbinnedBufs& B, const Mat& M, int64_t N, const double* h,
                const int64_t* Nk, const double* f, double* f_out, double* logD_out,
                double* lnS_out, double* S_out, SweepScalars* dev_scal, bool consts_ready,
                double* cst_next) {
  return queue_sweep(ctx, B, M, N, h, Nk, f, f_out, logD_out, lnS_out, S_out, dev_scal, false,
                     consts_ready, cst_next);
}

int sweep_at(bumbar_ctx* ctx, const UnbinnedBufs& B, const Mat& M, int64_t N, const double* h,
             const int64_t* Nk, const double* f, double* f_out, double* logD_out,
             double* lnS_out, double* S_out, SweepScalars* sc, bool force_robust,
             SweepCounters* cnt) {
  hipStream_t s = ctx->stream;
  const int K = B.K;
  SweepScalars tmp;
  SweepScalars* out = sc ? sc : &tmp;
  if (!force_robust || M.kind >= 2) {
    int rc = queue_sweep(ctx, B, M, N, h, Nk, f, f_out, logD_out, lnS_out, S_out, B.scal, true);
    if (rc) return rc;
    if (cnt) cnt->fast++;
    // callers without scalars still need the flags for the fallback decision
    rc = read_scalars(ctx, B.scal, out);
    if (rc) return rc;
    // FP32 kinds: flags are the caller's signal to leave FP32
    if (M.kind == 2 || M.kind == 3 || M.kind == 7) return BUMBAR_OK;
    if ((out->flags & (FLAG_COL | FLAG_STATE | FLAG_NAN)) == 0) {
      if (cnt && M.kind == 4 && M.otf.sep) cnt->grid++;
      return BUMBAR_OK;
    }
    if (M.kind == 4 && M.otf.sep) {
      // the product-grid passes shift by per-axis maxima: redo the sweep
      // with the direct passes
      Mat M2 = M;
      M2.otf.sep = nullptr;
      return sweep_at(ctx, B, M2, N, h, Nk, f, f_out, logD_out, lnS_out, S_out, sc, force_robust,
                      cnt);
    }
    if (M.kind == 4) {
      // the model sweep keeps exact maxima per sample; there is no separate
      // robust pass for it
      if (out->flags & FLAG_NAN) return fail(ctx, BUMBAR_EINVAL, "non-finite coordinates");
      return fail(ctx, BUMBAR_EINVAL,
                  "state or sample sums out of the FP64 range in the on-the-fly sweep");
    }
  }
  hipError_t e = launch_prepare_consts(s, K, Nk, f, B.cst, B.gk, B.lnNp);
  if (e != hipSuccess) return hip_fail(ctx, e, "prepare_consts");
  const int ch = robust_chunks(N);
  e = launch_sweep_robust(s, M.ut ? M.ut : M.u, M.ut ? M.ut_f32 : M.kind == 1,
                          M.ut ? smaj_row(K) : M.ld, K, N,
                          B.cst, B.gk, h, logD_out, B.part, B.partS, B.part_obj, B.part_flags, ch,
                          M.ut != nullptr);
  if (e != hipSuccess) return hip_fail(ctx, e, "sweep_robust");
  e = launch_sweep_finalize(s, 1, K, ch, B.part, B.partS, B.part_obj, B.part_flags, f, B.lnNp, Nk,
                            f_out, lnS_out, S_out, B.scal);
  if (e != hipSuccess) return hip_fail(ctx, e, "sweep_finalize");
  if (cnt) cnt->robust++;
  int rc = read_scalars(ctx, B.scal, out);
  if (rc) return rc;
  if (out->flags & FLAG_NAN)
    return fail(ctx, BUMBAR_EINVAL, "non-finite reduced energies (NaN or -inf in u_kn)");
  return BUMBAR_OK;
}

static hipError_t queue_hessian(bumbar_ctx* ctx, UnbinnedBufs& B, const Mat& M, const double* f) {
  // B.cst / B.gk hold the constants at f; the packed matrix needs d = f - f0
  // instead of c, and the model kinds their coefficients rebuilt at f.
  hipStream_t s = ctx->stream;
  const int hk = M.hess_kind >= 0 ? M.hess_kind : M.kind;
  HessSource hs;
  hs.kind = hk;
  hs.num_cus = ctx->num_cus;
  hs.u = M.u;
  hs.ld = M.ld;
  hs.otf = M.otf;
  hs.p16 = M.p16;
  const double* cst = B.cst;
  hipError_t e = hipSuccess;
  if (hk == 2) {
    e = launch_delta(s, B.K, f, M.f0, B.dk);
    hs.m0 = M.m0;
    cst = B.dk;
  } else if (hk == 3 || hk == 4) {
    // the model kinds: per-sweep coefficients at f
    e = launch_otf_coefs(s, M.otf, hk == 3, B.K, B.cst, B.gk);
  }
  if (e != hipSuccess) return e;
  return launch_hessian(s, hs, B.K, B.N, cst, B.gk, B.logD, B.S, B.hess_parts, B.hess_chunks,
                        B.H);
}

// Newton finisher on unbinned data (Section 2, derivative-based strategies).
// Each step solves the reduced Newton system and tries alpha = 1, 1/2, ...,
// 2^-10, accepting the first trial that lowers ||S - N||_2; if none does, one
// SCI step is taken. Convergence is declared only on a full Newton step:
// when a step with alpha = 1 is accepted and its max |delta f| < tol, or when
// the full step of a freshly built Hessian is itself below tol (then f is
// within about that distance of the fixed point, which is where the gradient
// norm stops falling at the rounding floor). A damped or SCI step says
// nothing about the distance to the solution (SCI contracts slowly where
// states overlap poorly), so the loop continues after one whatever its size.
// f (device, K) is updated in place.
//
// Work per step: the sweep at the accepted trial point doubles as the sweep
// at the new iterate (its ln D, S and constants are kept), and the Hessian is
// reused (a chord step) while the steps it gives keep halving the gradient
// norm; a stale Hessian that fails that test is rebuilt at the current f
// before any smaller trial is tried. Only the gradient, the line-search test
// and the stopping test need the matrix of M, so the fixed point reached is
// the one of M whatever Hessian produced the steps. B.H_valid carries a
// Hessian across calls (the FP64 refinement after the packed stage starts
// from the packed stage's Hessian). With the packed matrix, a flagged sweep
// ends the loop early with BUMBAR_ENOTCONV (the caller continues in FP64).
int newton_finish(bumbar_ctx* ctx, UnbinnedBufs& B, const Mat& M, const int64_t* Nk, double tol,
                  int max_steps, bumbar_stats* st, SweepCounters* cnt, double* final_step,
                  double* final_gnorm) {
  hipStream_t s = ctx->stream;
  const int K = B.K;
  const int64_t N = B.N;
  SweepScalars sc{};
  const bool fp32 = M.kind == 2 || M.kind == 3 || M.kind == 7;
  auto bad32 = [&](const SweepScalars& x) {
    return fp32 && (x.flags & (FLAG_COL | FLAG_STATE | FLAG_NAN)) != 0;
  };
  // the sweep at the starting point; unsampled states filled and the gauge
  // fixed afterwards (neither changes S of sampled states, ln D - c or the
  // gradient norm, so the sweep stays the sweep at f)
  int rc = sweep_at(ctx, B, M, N, nullptr, Nk, B.f, B.f_new, B.logD, B.lnS, B.S, &sc, false, cnt);
  if (rc) return rc;
  if (bad32(sc)) return BUMBAR_ENOTCONV;
  // B.cst and B.logD must describe the same point when the Hessian is built
  // from them: the trial sweeps overwrite B.cst, and the gauge shift moves f
  // after its sweep, so the constants are rebuilt at the swept point f_sweep.
  hipError_t e = hipMemcpyAsync(B.f_sweep, B.f, sizeof(double) * K, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = launch_fill_unsampled_gauge(s, K, Nk, B.f, B.lnS);
  if (e != hipSuccess) return hip_fail(ctx, e, "fill_unsampled");
  auto build_hessian = [&]() -> int {
    hipError_t e2 = launch_prepare_consts(s, K, Nk, B.f_sweep, B.cst, B.gk, B.lnNp);
    if (e2 == hipSuccess) e2 = queue_hessian(ctx, B, M, B.f_sweep);
    if (e2 != hipSuccess) return hip_fail(ctx, e2, "hessian");
    if (st) st->hessians++;
    B.H_valid = true;
    return BUMBAR_OK;
  };
  auto direction = [&](int* ok) -> int {
    hipError_t e2 = (B.m_red > newton_lds_max_m())
                        ? launch_newton_direction_blocked(s, K, B.m_red, Nk, B.H, B.S, B.A, B.idx,
                                                          B.dir, B.ok)
                        : launch_newton_direction(s, K, Nk, B.H, B.S, B.A, B.idx, B.dir, B.ok);
    if (e2 != hipSuccess) return hip_fail(ctx, e2, "newton_direction");
    return read_bytes(ctx, B.ok, ok, sizeof(int));
  };
  int steps = 0, fallbacks = 0, damped = 0;
  double last = INFINITY;
  rc = BUMBAR_ENOTCONV;
  while (steps < max_steps) {
    const double gn = sc.grad_norm;
    if (final_gnorm) *final_gnorm = gn;
    bool fresh = false;
    if (!B.H_valid) {
      rc = build_hessian();
      if (rc) return rc;
      fresh = true;
    }
    bool accepted = false, flagged = false, full = false;
    bool fresh_dir = false;  // the last direction came from a freshly built Hessian
    SweepScalars st2{};
    for (;;) {
      int ok = 0;
      rc = direction(&ok);
      if (rc) return rc;
      if (!ok && !fresh) {
        rc = build_hessian();
        if (rc) return rc;
        fresh = true;
        continue;
      }
      if (!ok) break;
      fresh_dir = fresh;
      double alpha = 1.0;
      // FP32 kinds take full steps only: below the FP32 resolution the
      // gradient norm stops falling and the FP64 refinement takes over
      const int max_t = fp32 ? 0 : 10;
      for (int t = 0; t <= max_t; ++t, alpha *= 0.5) {
        e = launch_axpy_to(s, K, B.f, alpha, B.dir, B.f_trial);
        // the full step's size (read back only if no trial is accepted)
        if (e == hipSuccess && t == 0) e = launch_max_abs_diff(s, K, B.f_trial, B.f, B.misc + 1);
        if (e != hipSuccess) return hip_fail(ctx, e, "axpy");
        rc = sweep_at(ctx, B, M, N, nullptr, Nk, B.f_trial, B.f_new, B.logD_t, B.lnS_t, B.S_t,
                      &st2, false, cnt);
        if (rc) return rc;
        if (bad32(st2)) {
          flagged = true;
          break;
        }
        // a stale Hessian must at least halve the gradient norm at alpha = 1
        if (fresh ? st2.grad_norm < gn : st2.grad_norm < 0.5 * gn) {
          accepted = true;
          full = t == 0;
          break;
        }
        if (!fresh) break;
      }
      // a stale Hessian that fails is rebuilt, except in the FP32 kinds: there
      // the failure means the FP32 noise floor, and the FP64 stage takes over
      if (accepted || flagged || fresh || fp32) break;
      rc = build_hessian();
      if (rc) return rc;
      fresh = true;
    }
    if (flagged || (fp32 && !accepted)) {
      rc = BUMBAR_ENOTCONV;
      break;
    }
    if (!accepted && fresh_dir) {
      // the full step of a fresh Hessian below tol: f is already that close
      // to the fixed point (the gradient norm no longer falls: rounding floor)
      double full_step = INFINITY;
      rc = read_bytes(ctx, B.misc + 1, &full_step, sizeof(double));
      if (rc) return rc;
      if (full_step < tol) {
        last = full_step;
        rc = BUMBAR_OK;
        break;
      }
    }
    if (accepted && !full) ++damped;
    if (!accepted) {
      // SCI step from the sweep at f: f_trial = SCI(f) (gauged), then the
      // sweep at f_trial
      rc = sweep_at(ctx, B, M, N, nullptr, Nk, B.f, B.f_trial, B.logD_t, B.lnS_t, B.S_t, nullptr,
                    false, cnt);
      if (rc) return rc;
      rc = sweep_at(ctx, B, M, N, nullptr, Nk, B.f_trial, B.f_new, B.logD_t, B.lnS_t, B.S_t, &st2,
                    false, cnt);
      if (rc) return rc;
      if (bad32(st2)) {
        rc = BUMBAR_ENOTCONV;
        break;
      }
      ++fallbacks;
    }
    e = hipMemcpyAsync(B.f_sweep, B.f_trial, sizeof(double) * K, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = launch_fill_unsampled_gauge(s, K, Nk, B.f_trial, B.lnS_t);
    if (e != hipSuccess) return hip_fail(ctx, e, "fill_unsampled");
    e = launch_max_abs_diff(s, K, B.f_trial, B.f, B.misc);
    if (e != hipSuccess) return hip_fail(ctx, e, "max_abs_diff");
    // the trial point becomes the iterate, its sweep the sweep at f
    std::swap(B.f, B.f_trial);
    std::swap(B.logD, B.logD_t);
    std::swap(B.lnS, B.lnS_t);
    std::swap(B.S, B.S_t);
    sc = st2;
    rc = read_bytes(ctx, B.misc, &last, sizeof(double));
    if (rc) return rc;
    ++steps;
    if (final_gnorm) *final_gnorm = sc.grad_norm;
    // only a full Newton step bounds the remaining error
    if (full && last < tol) {
      rc = BUMBAR_OK;
      break;
    }
    rc = BUMBAR_ENOTCONV;
  }
  if (st) {
    st->finisher_steps += steps;
    st->sci_fallbacks += fallbacks;
    st->damped_steps += damped;
  }
  if (final_step) *final_step = last;
  return rc;
}

// Plain self-consistent iteration on unbinned data until the step is below
// `until` (or the cap); f updated in place.
int sci_until(bumbar_ctx* ctx, UnbinnedBufs& B, const Mat& M, const int64_t* Nk, double until,
              int64_t max_steps, int64_t* steps_out, SweepCounters* cnt, double* last_step) {
  SweepScalars sc{};
  int64_t it = 0;
  int rc = BUMBAR_ENOTCONV;
  while (it < max_steps) {
    rc = sweep_at(ctx, B, M, B.N, nullptr, Nk, B.f, B.f_new, B.logD, B.lnS, B.S, &sc, false, cnt);
    if (rc) return rc;
    hipError_t e =
        hipMemcpyAsync(B.f, B.f_new, sizeof(double) * B.K, hipMemcpyDeviceToDevice, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "copy f");
    ++it;
    if (last_step) *last_step = sc.max_df;
    if (sc.max_df < until) {
      rc = BUMBAR_OK;
      break;
    }
    rc = BUMBAR_ENOTCONV;
  }
  if (steps_out) *steps_out = it;
  return rc;
}

}  // namespace bumbar

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

#ifndef BUMBAR_SOURCE_HASH
#define BUMBAR_SOURCE_HASH "unknown"
#endif
const char* bumbar_version(void) { return "bumbar-gfx950 0.2 src:" BUMBAR_SOURCE_HASH; }

int bumbar_create(bumbar_ctx** out, int device, void* hip_stream) {
  if (!out) return BUMBAR_EINVAL;
  *out = nullptr;
  bumbar_ctx* c = new (std::nothrow) bumbar_ctx();
  if (!c) return BUMBAR_ENOMEM;
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) {
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, device);
    if (e == hipSuccess) c->num_cus = p.multiProcessorCount;
  }
  if (e == hipSuccess) e = hipHostMalloc(&c->pinned, kPinnedBytes, hipHostMallocDefault);
  if (e != hipSuccess || static_scratch_init(c) != BUMBAR_OK) {
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
    return BUMBAR_EDEVICE;
  }
  *out = c;
  return BUMBAR_OK;
}

void bumbar_destroy(bumbar_ctx* ctx) {
  if (!ctx) return;
  for (auto& p : ctx->events) {
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
}

const char* bumbar_last_error(const bumbar_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

void bumbar_default_options(bumbar_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-10;
  o->precision = BUMBAR_PREC_FP64;
  o->binning = 0;
  o->n0 = 100;
  o->eps = 1e-3;
  o->inc = 10;
  o->n_intermediate = 20;
  o->finisher = BUMBAR_FINISH_NEWTON;
  o->max_iter = 1000000;
  o->max_newton = 100;
  o->sci_switch = 1e-3;
  o->replay_phase1 = 0;
  o->replay_refine = nullptr;
  o->n_replay = 0;
  o->profile = 0;
  o->mixed_tol = 1e-6;
  o->represent = BUMBAR_REPRESENT_AUTO;
  o->graphs = 1;
  o->sample_major = 1;
  o->u_dtype = BUMBAR_F64;
  o->xi_dtype = BUMBAR_F64;
  o->grid_batches = 0;
}

static int check_common(bumbar_ctx* ctx, const void* u, int u_dtype, int K, int64_t N,
                        int64_t ld, bool smaj_ok = false) {
  if (!ctx) return BUMBAR_EINVAL;
  ctx->err.clear();
  if (!u) return fail(ctx, BUMBAR_EINVAL, "u_kn is NULL");
  if (K <= 0 || N <= 0) return fail(ctx, BUMBAR_EINVAL, "K and N must be positive");
  const bool smaj = u_dtype == BUMBAR_F64_SMAJOR || u_dtype == BUMBAR_F32_SMAJOR;
  if (smaj) {
    if (!smaj_ok) return fail(ctx, BUMBAR_EINVAL, "this call takes state-major u_kn only");
    if (!sweep_smaj_supported(K))
      return fail(ctx, BUMBAR_EINVAL, "the sample-major layout is defined for 256 < K <= 1024");
  } else {
    if (ld < N) return fail(ctx, BUMBAR_EINVAL, "row stride ld < N");
    if (u_dtype != BUMBAR_F64 && u_dtype != BUMBAR_F32)
      return fail(ctx, BUMBAR_EINVAL, "u_dtype must be BUMBAR_F64 or BUMBAR_F32");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BUMBAR_EDEVICE, "hipSetDevice");
  return BUMBAR_OK;
}

static Mat input_mat(const void* u, int u_dtype, int64_t ld) {
  Mat M;
  M.u = u;
  M.kind = (u_dtype == BUMBAR_F32 || u_dtype == BUMBAR_F32_SMAJOR) ? 1 : 0;
  M.ld = ld;
  if (u_dtype == BUMBAR_F64_SMAJOR || u_dtype == BUMBAR_F32_SMAJOR) {
    M.ut = u;
    M.ut_f32 = u_dtype == BUMBAR_F32_SMAJOR;
  }
  return M;
}

int64_t bumbar_sample_major_elems(int K, int64_t N) {
  if (!sweep_smaj_supported(K) || N <= 0) return -1;
  return (int64_t)smaj_elems(K, N);
}

int bumbar_sample_major(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N,
                        int64_t ld, void* u_nk) {
  int rc = check_common(ctx, u_kn, u_dtype, K, N, ld);
  if (rc) return rc;
  if (!sweep_smaj_supported(K))
    return fail(ctx, BUMBAR_EINVAL, "the sample-major layout is defined for 256 < K <= 1024");
  if (!u_nk) return fail(ctx, BUMBAR_EINVAL, "NULL output");
  const hipError_t e =
      launch_smaj_copy(ctx->stream, u_kn, u_dtype == BUMBAR_F32, ld, K, N, u_nk, nullptr);
  if (e != hipSuccess) return hip_fail(ctx, e, "sample-major copy");
  return BUMBAR_OK;
}

int bumbar_sweep(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N, int64_t ld,
                 const int64_t* N_k, const double* f, void* workspace, size_t ws_bytes,
                 double* f_new, double* log_D_n, double* S, double* sweep_stats) {
  const bool smaj = u_dtype == BUMBAR_F64_SMAJOR || u_dtype == BUMBAR_F32_SMAJOR;
  if (smaj) ld = N;
  int rc = check_common(ctx, u_kn, u_dtype, K, N, ld, true);
  if (rc) return rc;
  if (!N_k || !f || !f_new || !workspace) return fail(ctx, BUMBAR_EINVAL, "NULL argument");
  Arena ar{reinterpret_cast<char*>(workspace), ws_bytes};
  UnbinnedBufs B;
  B.carve(ar, K, N, ctx->num_cus);
  if (ar.overflow) return fail(ctx, BUMBAR_ENOMEM, "workspace too small (%zu bytes)", ws_bytes);
  double* logD = log_D_n ? log_D_n : B.logD;
  double* Sv = S ? S : B.S;
  SweepScalars sc{};
  const Mat M = input_mat(u_kn, u_dtype, ld);
  if (sweep_stats == nullptr && ((M.kind <= 1 && sweep_fast_supported(K)) || M.ut)) {
    // asynchronous: queue the sweep without reading anything back (the caller
    // accepts that a far-off f is not rerun on the robust path)
    return sweep_queue(ctx, B, M, N, nullptr, N_k, f, f_new, logD, B.lnS, Sv, B.scal);
  }
  rc = sweep_at(ctx, B, M, N, nullptr, N_k, f, f_new, logD, B.lnS, Sv, &sc, false, nullptr);
  if (rc) return rc;
  if (sweep_stats) {
    sweep_stats[0] = sc.max_df;
    sweep_stats[1] = sc.rel_step;
    sweep_stats[2] = sc.objective;
    sweep_stats[3] = sc.grad_norm;
  }
  return BUMBAR_OK;
}

int bumbar_hessian(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N,
                   int64_t ld, const int64_t* N_k, const double* f, const double* log_D_n,
                   const double* S, void* workspace, size_t ws_bytes, double* H) {
  int rc = check_common(ctx, u_kn, u_dtype, K, N, ld);
  if (rc) return rc;
  if (!N_k || !f || !log_D_n || !S || !H || !workspace)
    return fail(ctx, BUMBAR_EINVAL, "NULL argument");
  Arena ar{reinterpret_cast<char*>(workspace), ws_bytes};
  UnbinnedBufs B;
  B.carve(ar, K, N, ctx->num_cus);
  if (ar.overflow) return fail(ctx, BUMBAR_ENOMEM, "workspace too small");
  hipError_t e = launch_prepare_consts(ctx->stream, K, N_k, f, B.cst, B.gk, B.lnNp);
  HessSource hs;
  hs.kind = u_dtype == BUMBAR_F32 ? 1 : 0;
  hs.u = u_kn;
  hs.ld = ld;
  if (e == hipSuccess)
    e = launch_hessian(ctx->stream, hs, K, N, B.cst, B.gk, log_D_n, S, B.hess_parts,
                       B.hess_chunks, H);
  if (e != hipSuccess) return hip_fail(ctx, e, "hessian");
  return BUMBAR_OK;
}

int bumbar_hessian_fp16(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N,
                        int64_t ld, const int64_t* N_k, const double* f, const double* log_D_n,
                        const double* S, void* workspace, size_t ws_bytes, double* H) {
  int rc = check_common(ctx, u_kn, u_dtype, K, N, ld);
  if (rc) return rc;
  if (K <= 256) return fail(ctx, BUMBAR_EINVAL, "the FP16-core Hessian takes K > 256");
  if (u_dtype != BUMBAR_F64 && u_dtype != BUMBAR_F32)
    return fail(ctx, BUMBAR_EINVAL, "u_dtype must be BUMBAR_F64 or BUMBAR_F32");
  if (!N_k || !f || !log_D_n || !S || !H || !workspace)
    return fail(ctx, BUMBAR_EINVAL, "NULL argument");
  Arena ar{reinterpret_cast<char*>(workspace), ws_bytes};
  UnbinnedBufs B;
  B.carve(ar, K, N, ctx->num_cus);
  char* p16 = ar.take<char>((size_t)K * (size_t)p16_samples(K, N) * 2);
  if (ar.overflow) return fail(ctx, BUMBAR_ENOMEM, "workspace too small");
  hipError_t e = launch_prepare_consts(ctx->stream, K, N_k, f, B.cst, B.gk, B.lnNp);
  HessSource hs;
  hs.kind = u_dtype == BUMBAR_F32 ? 8 : 5;
  hs.num_cus = ctx->num_cus;
  hs.u = u_kn;
  hs.ld = ld;
  hs.p16 = p16;
  if (e == hipSuccess)
    e = launch_hessian(ctx->stream, hs, K, N, B.cst, B.gk, log_D_n, S, B.hess_parts,
                       B.hess_chunks, H);
  if (e != hipSuccess) return hip_fail(ctx, e, "hessian");
  return BUMBAR_OK;
}

static void carve_cov(Arena& ar, UnbinnedBufs& B, int K, int64_t N, int num_cus, double** Th,
                      double** Bm) {
  B.carve(ar, K, N, num_cus);
  *Th = ar.take<double>((size_t)K * K);
  *Bm = ar.take<double>((size_t)K * K);
}

int bumbar_query_workspace_covariance(const bumbar_ctx* ctx, int K, int64_t N, size_t* bytes) {
  if (!ctx || !bytes || K <= 0 || N <= 0) return BUMBAR_EINVAL;
  Arena ar;
  UnbinnedBufs B;
  double *Th, *Bm;
  carve_cov(ar, B, K, N, ctx->num_cus, &Th, &Bm);
  *bytes = ar.off + 256;
  return BUMBAR_OK;
}

int bumbar_covariance(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N,
                      int64_t ld, const int64_t* N_k, const double* f, void* workspace,
                      size_t ws_bytes, double* cov) {
  int rc = check_common(ctx, u_kn, u_dtype, K, N, ld);
  if (rc) return rc;
  if (!N_k || !f || !cov || !workspace) return fail(ctx, BUMBAR_EINVAL, "NULL argument");
  std::vector<int64_t> nk(K);
  rc = read_bytes(ctx, N_k, nk.data(), sizeof(int64_t) * K);
  if (rc) return rc;
  int64_t tot = 0;
  std::vector<int> kept;  // sampled states but the first: the reduced system
  for (int k = 0, first = 1; k < K; ++k) {
    if (nk[k] < 0) return fail(ctx, BUMBAR_EINVAL, "negative N_k");
    tot += nk[k];
    if (nk[k] > 0) {
      if (!first) kept.push_back(k);
      first = 0;
    }
  }
  if (tot != N) return fail(ctx, BUMBAR_EINVAL, "sum of N_k (%lld) != N (%lld)", (long long)tot,
                            (long long)N);
  Arena ar{reinterpret_cast<char*>(workspace), ws_bytes};
  UnbinnedBufs B;
  double *Th, *Bm;
  carve_cov(ar, B, K, N, ctx->num_cus, &Th, &Bm);
  if (ar.overflow)
    return fail(ctx, BUMBAR_ENOMEM, "workspace too small (%zu bytes, need %zu)", ws_bytes, ar.off);
  hipStream_t s = ctx->stream;
  // ln D_n at f by one unbinned sweep
  Mat M = input_mat(u_kn, u_dtype, ld);
  SweepScalars sc{};
  rc = sweep_at(ctx, B, M, N, nullptr, N_k, f, B.f_new, B.logD, B.lnS, B.S, &sc, false, nullptr);
  if (rc) return rc;
  // -M = -W^T W from the Hessian contraction with P = W
  hipError_t e = launch_cov_consts(s, K, f, B.cst, B.gk, B.S);
  HessSource hs;
  hs.kind = M.kind;
  hs.u = u_kn;
  hs.ld = ld;
  if (e == hipSuccess)
    e = launch_hessian(s, hs, K, N, B.cst, B.gk, B.logD, B.S, B.hess_parts, B.hess_chunks, B.H);
  const int m = (int)kept.size();
  double* b = B.A + (int64_t)m * m;
  double* y = b + m;
  double* Linv = y + m;
  if (e == hipSuccess && m > 0)
    e = hipMemcpyAsync(B.idx, kept.data(), sizeof(int) * m, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && m > 0) e = launch_cov_gather(s, K, m, B.idx, N_k, B.H, B.A, b, Bm);
  if (e == hipSuccess && m > 0) e = launch_chol_factor_blocked(s, m, B.A, b, y, Linv, B.ok);
  if (e != hipSuccess) return hip_fail(ctx, e, "covariance");
  if (m > 0) {
    int ok = 0;
    rc = read_bytes(ctx, B.ok, &ok, sizeof(int));
    if (rc) return rc;
    if (!ok)
      return fail(ctx, BUMBAR_EINVAL,
                  "the reduced Hessian is not positive definite (states without overlap)");
    e = launch_cov_solve(s, m, K, B.A, Linv, Bm);
  }
  if (e == hipSuccess) e = launch_cov_theta(s, m, K, Bm, B.H, Th, cov);
  if (e == hipSuccess) e = ctx_wait(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "covariance");
  return BUMBAR_OK;
}

// Product-grid detection for the 2-D harmonic model (host side, once per
// call): the distinct (kappa_x / 2, x0) and (kappa_y / 2, y0) pairs of the K
// states. The factored FP64 sweep is used when each axis has at most kSepMax
// of them and the two together at most K / 4 (below that it saves little).
// g receives the device arrays in O (filled here); *on says whether to use it.
static int sep_setup(bumbar_ctx* ctx, int K, int d, int model, const double* coef,
                     const OtfBufs& O, SepGrid* g, bool* on) {
  *on = false;
  if (d != 2 || model != BUMBAR_MODEL_HARMONIC || !O.sep_i || !O.sep_d || K < 16)
    return BUMBAR_OK;
  std::vector<double> c((size_t)K * 5);
  int rc = read_bytes(ctx, coef, c.data(), sizeof(double) * c.size());
  if (rc) return rc;
  std::map<std::pair<double, double>, int> xs, ys;
  std::vector<int> ibuf(sep_int_count(K), 0);
  std::vector<double> dbuf(4 * kSepMax, 0.0);
  int* ix = ibuf.data();
  int* jy = ix + K;
  int* cstates = jy + K;
  int* cstart = cstates + K;
  for (int k = 0; k < K; ++k) {
    const double* ck = c.data() + (size_t)k * 5;
    for (int t = 1; t < 5; ++t)
      if (!std::isfinite(ck[t])) return BUMBAR_OK;
    const std::pair<double, double> px{0.5 * ck[1], ck[2]}, py{0.5 * ck[3], ck[4]};
    auto itx = xs.find(px);
    if (itx == xs.end()) {
      if ((int)xs.size() == kSepMax) return BUMBAR_OK;
      const int i = (int)xs.size();
      dbuf[2 * i] = px.first;
      dbuf[2 * i + 1] = px.second;
      itx = xs.emplace(px, i).first;
    }
    auto ity = ys.find(py);
    if (ity == ys.end()) {
      if ((int)ys.size() == kSepMax) return BUMBAR_OK;
      const int j = (int)ys.size();
      dbuf[2 * kSepMax + 2 * j] = py.first;
      dbuf[2 * kSepMax + 2 * j + 1] = py.second;
      ity = ys.emplace(py, j).first;
    }
    ix[k] = itx->second;
    jy[k] = ity->second;
  }
  const int Ix = (int)xs.size(), Jy = (int)ys.size();
  if (4 * (Ix + Jy) > K) return BUMBAR_OK;
  // cells c = i * Jy + j, their states in increasing k
  for (int k = 0; k < K; ++k) ++cstart[ix[k] * Jy + jy[k] + 1];
  for (int q = 0; q < Ix * Jy; ++q) cstart[q + 1] += cstart[q];
  std::vector<int> cur(cstart, cstart + Ix * Jy);
  for (int k = 0; k < K; ++k) cstates[cur[ix[k] * Jy + jy[k]]++] = k;
  hipError_t e = hipMemcpyAsync(O.sep_i, ibuf.data(), sizeof(int) * ibuf.size(),
                                hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(O.sep_d, dbuf.data(), sizeof(double) * dbuf.size(),
                       hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = ctx_wait(ctx, ctx->stream);  // the host buffers end here
  if (e != hipSuccess) return hip_fail(ctx, e, "upload product grid");
  g->Ix = Ix;
  g->Jy = Jy;
  g->JM = (Jy + 7) / 8 * 8;
  g->fx = O.sep_d;
  g->fy = O.sep_d + 2 * kSepMax;
  g->C = O.sep_d + 4 * kSepMax;
  g->cmax = g->C + kSepMax * kSepMax;
  g->ix = O.sep_i;
  g->jy = O.sep_i + K;
  g->cstates = O.sep_i + 2 * K;
  g->cstart = O.sep_i + 3 * K;
  *on = true;
  return BUMBAR_OK;
}

// Model problem of K states over N coordinates: the on-the-fly kinds.
static int model_setup(bumbar_ctx* ctx, int K, int64_t N, int d, int model, const double* coef,
                       const double* xi, int precision, void* workspace, size_t ws_bytes,
                       UnbinnedBufs* B, Mat* M, SepGrid* sg = nullptr) {
  int rc = check_common(ctx, coef, BUMBAR_F64, K, N, N);
  if (rc) return rc;
  if ((model != BUMBAR_MODEL_LINEAR && model != BUMBAR_MODEL_HARMONIC) || !xi || d < 1 || d > 2)
    return fail(ctx, BUMBAR_EINVAL, "needs a LINEAR or HARMONIC model and xi with d in {1, 2}");
  if (precision != BUMBAR_PREC_FP64 && precision != BUMBAR_PREC_MIXED)
    return fail(ctx, BUMBAR_EINVAL, "unknown precision");
  if (!workspace) return fail(ctx, BUMBAR_EINVAL, "NULL workspace");
  Arena ar{reinterpret_cast<char*>(workspace), ws_bytes};
  B->carve(ar, K, N, ctx->num_cus);
  OtfBufs O;
  O.carve(ar, K, N, d);
  // the FP32 model's Hessian on the FP16 matrix cores reads a tiled FP16 copy of P
  if (precision == BUMBAR_PREC_MIXED && K > 256)
    M->p16 = ar.take<char>((size_t)K * (size_t)p16_samples(K, N) * 2);
  if (ar.overflow) return fail(ctx, BUMBAR_ENOMEM, "workspace too small (%zu bytes)", ws_bytes);
  M->kind = precision == BUMBAR_PREC_MIXED ? 3 : 4;
  M->otf.xi = xi;
  M->otf.xf = O.xf;
  M->otf.coef = coef;
  M->otf.d = d;
  M->otf.model = model;
  M->otf.cf32 = O.cf32;
  M->otf.cf64 = O.cf64;
  if (M->kind == 3) {
    const hipError_t e = launch_pack_coords(ctx->stream, N * d, xi, O.xf);
    if (e != hipSuccess) return hip_fail(ctx, e, "pack coordinates");
  }
  if (sg) {
    bool on = false;
    rc = sep_setup(ctx, K, d, model, coef, O, sg, &on);
    if (rc) return rc;
    if (on) M->otf.sep = sg;
  }
  return BUMBAR_OK;
}

int bumbar_sweep_model(bumbar_ctx* ctx, int K, int64_t N, int d, int model, const double* coef,
                       const double* xi, int precision, const int64_t* N_k, const double* f,
                       void* workspace, size_t ws_bytes, double* f_new, double* log_D_n,
                       double* S, double* sweep_stats) {
  UnbinnedBufs B;
  Mat M;
  SepGrid sg;
  int rc = model_setup(ctx, K, N, d, model, coef, xi, precision, workspace, ws_bytes, &B, &M, &sg);
  if (rc) return rc;
  if (!N_k || !f || !f_new) return fail(ctx, BUMBAR_EINVAL, "NULL argument");
  SweepScalars sc{};
  rc = sweep_at(ctx, B, M, N, nullptr, N_k, f, f_new, log_D_n ? log_D_n : B.logD, B.lnS,
                S ? S : B.S, &sc, false, nullptr);
  if (rc) return rc;
  if (M.kind == 3 && (sc.flags & (FLAG_COL | FLAG_STATE | FLAG_NAN)))
    return fail(ctx, BUMBAR_EINVAL, "sums out of the FP32 range in the FP32 model sweep");
  if (sweep_stats) {
    sweep_stats[0] = sc.max_df;
    sweep_stats[1] = sc.rel_step;
    sweep_stats[2] = sc.objective;
    sweep_stats[3] = sc.grad_norm;
  }
  return BUMBAR_OK;
}

int bumbar_hessian_model(bumbar_ctx* ctx, int K, int64_t N, int d, int model, const double* coef,
                         const double* xi, int precision, const int64_t* N_k, const double* f,
                         const double* log_D_n, const double* S, void* workspace,
                         size_t ws_bytes, double* H) {
  UnbinnedBufs B;
  Mat M;
  int rc = model_setup(ctx, K, N, d, model, coef, xi, precision, workspace, ws_bytes, &B, &M);
  if (rc) return rc;
  if (!N_k || !f || !log_D_n || !S || !H) return fail(ctx, BUMBAR_EINVAL, "NULL argument");
  hipError_t e = launch_prepare_consts(ctx->stream, K, N_k, f, B.cst, B.gk, B.lnNp);
  HessSource hs;
  hs.kind = M.kind;
  hs.num_cus = ctx->num_cus;
  hs.otf = M.otf;
  hs.p16 = M.p16;
  if (e == hipSuccess) e = launch_otf_coefs(ctx->stream, M.otf, M.kind == 3, K, B.cst, B.gk);
  if (e == hipSuccess)
    e = launch_hessian(ctx->stream, hs, K, N, B.cst, B.gk, log_D_n, S, B.hess_parts,
                       B.hess_chunks, H);
  if (e != hipSuccess) return hip_fail(ctx, e, "hessian");
  return BUMBAR_OK;
}

int bumbar_weights(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N, int64_t ld,
                   const double* f, const double* log_D_n, double* W_nk) {
  int rc = check_common(ctx, u_kn, u_dtype, K, N, ld);
  if (rc) return rc;
  if (!f || !log_D_n || !W_nk) return fail(ctx, BUMBAR_EINVAL, "NULL argument");
  hipError_t e = launch_weights(ctx->stream, u_kn, u_dtype == BUMBAR_F32, ld, K, N, f, log_D_n,
                                W_nk);
  if (e != hipSuccess) return hip_fail(ctx, e, "weights");
  return BUMBAR_OK;
}

int bumbar_reweight(bumbar_ctx* ctx, const double* u_target, int64_t N, const double* log_D_n,
                    void* workspace, size_t ws_bytes, double* p) {
  if (!ctx) return BUMBAR_EINVAL;
  ctx->err.clear();
  if (!u_target || !log_D_n || !p || !workspace || N <= 0)
    return fail(ctx, BUMBAR_EINVAL, "bad argument");
  const int nparts = 1024;
  if (ws_bytes < sizeof(double) * (2 * nparts + 2))
    return fail(ctx, BUMBAR_ENOMEM, "workspace too small");
  hipError_t e = launch_reweight(ctx->stream, N, u_target, log_D_n,
                                 reinterpret_cast<double*>(workspace), nparts, p);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "reweight");
  return BUMBAR_OK;
}

int bumbar_model_energies(bumbar_ctx* ctx, int K, int64_t N, int d, int model,
                          const double* coef, const double* xi, int u_dtype, void* u_kn) {
  if (!ctx) return BUMBAR_EINVAL;
  ctx->err.clear();
  if (K <= 0 || N <= 0 || (d != 1 && d != 2) || !coef || !xi || !u_kn ||
      (model != BUMBAR_MODEL_LINEAR && model != BUMBAR_MODEL_HARMONIC) ||
      (u_dtype != BUMBAR_F64 && u_dtype != BUMBAR_F32))
    return fail(ctx, BUMBAR_EINVAL, "bad argument");
  const hipError_t e = launch_model_energies(ctx->stream, K, N, d, model, coef, xi, u_kn,
                                             u_dtype == BUMBAR_F32);
  if (e != hipSuccess) return hip_fail(ctx, e, "model energies");
  return BUMBAR_OK;
}

int bumbar_query_workspace(const bumbar_ctx* ctx, int K, int64_t N, int d,
                           const bumbar_options* opt, size_t* bytes) {
  if (!ctx || !bytes || K <= 0 || N <= 0 || d < 0 || d > 2) return BUMBAR_EINVAL;
  bumbar_options o;
  if (opt) {
    o = *opt;
    o.binning = o.binning && d > 0;
  } else {
    bumbar_default_options(&o);
    o.binning = d > 0;
  }
  Plan p;
  std::string why;
  if (make_plan(o, false, o.u_dtype, K, N, d, -1, &p, &why) != BUMBAR_OK) return BUMBAR_EINVAL;
  Arena ar;
  PlanBufs pb;
  carve_plan(ar, p, ctx->num_cus, &pb);
  *bytes = ar.off + 256;
  return BUMBAR_OK;
}

int bumbar_query_workspace_model(const bumbar_ctx* ctx, int K, int64_t N, int d,
                                 const bumbar_options* opt, size_t* bytes) {
  if (!ctx || !bytes || K <= 0 || N <= 0 || d < 1 || d > 2) return BUMBAR_EINVAL;
  bumbar_options o;
  if (opt) {
    o = *opt;
  } else {
    bumbar_default_options(&o);
    o.binning = 1;
  }
  // without options: enough for the solve at either precision (and so for
  // bumbar_sweep_model / bumbar_hessian_model at either)
  size_t most = 0;
  for (int pass = 0; pass < (opt ? 1 : 2); ++pass) {
    if (!opt) {
      o.precision = pass ? BUMBAR_PREC_MIXED : BUMBAR_PREC_FP64;
      o.finisher = BUMBAR_FINISH_NEWTON;
    }
    Plan p;
    std::string why;
    if (make_plan(o, true, BUMBAR_F64, K, N, d, BUMBAR_MODEL_HARMONIC, &p, &why) != BUMBAR_OK)
      return BUMBAR_EINVAL;
    Arena ar;
    PlanBufs pb;
    carve_plan(ar, p, ctx->num_cus, &pb);
    most = std::max(most, ar.off);
  }
  *bytes = most + 256;
  return BUMBAR_OK;
}

// The solve's trace: one line per phase-2 check of Algorithm 1 (nominal n,
// the bins at n and n inc, the relative steps of Eq. (2), the decision), then
// a summary line (stage lengths, finisher steps, last step, gradient norm,
// stage times). Text, appended to path; EINVAL if it cannot be written.
constexpr int kTraceChecks = 4096;
static int write_trace(bumbar_ctx* ctx, const char* path, int K, int64_t N, const bumbar_stats& st) {
  FILE* fp = std::fopen(path, "a");
  if (!fp) return fail(ctx, BUMBAR_EINVAL, "cannot open the trace file %s", path);
  std::fprintf(fp, "# bumbar trace K=%d N=%lld\n", K, (long long)N);
  std::fprintf(fp, "# check n P P_next s_n s_next refine stop\n");
  const int64_t n = std::min<int64_t>(st.n_checks, st.checks ? st.checks_capacity : 0);
  for (int64_t i = 0; i < n; ++i) {
    const bumbar_check& c = st.checks[i];
    std::fprintf(fp, "check %lld %lld %lld %lld %.17g %.17g %d %d\n", (long long)i, (long long)c.n,
                 (long long)c.P, (long long)c.P_next, c.s_n, c.s_next, c.refine, c.stop);
  }
  std::fprintf(fp,
               "summary phase1_iters=%lld phase2_iters=%lld n_checks=%lld finisher_steps=%lld "
               "sci_fallbacks=%lld unbinned_sweeps=%lld hessians=%lld mixed_steps=%lld "
               "final_step=%.17g grad_norm=%.17g time_binning_ms=%.6f time_binned_ms=%.6f "
               "time_final_ms=%.6f\n",
               (long long)st.phase1_iters, (long long)st.phase2_iters, (long long)st.n_checks,
               (long long)st.finisher_steps, (long long)st.sci_fallbacks,
               (long long)st.unbinned_sweeps, (long long)st.hessians, (long long)st.mixed_steps,
               st.final_step, st.grad_norm, st.time_binning_ms, st.time_binned_ms,
               st.time_final_ms);
  const bool ok = std::fclose(fp) == 0;
  return ok ? BUMBAR_OK : fail(ctx, BUMBAR_EINVAL, "cannot write the trace file %s", path);
}

int bumbar_solve(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N,
                 const int64_t* N_k, const void* xi_in, int xi_dtype, int d, int model,
                 const double* coef, const double* f_init, const bumbar_options* opt_in,
                 void* workspace, size_t ws_bytes, double* f_k, double* W_nk,
                 double* log_D_n, bumbar_stats* stats) {
  // u_kn == NULL: the energies come from the model, evaluated in the kernels
  const bool otf = (u_kn == nullptr);
  int rc = otf ? check_common(ctx, coef, BUMBAR_F64, K, N, N) : check_common(ctx, u_kn, u_dtype, K,
                                                                             N, N);
  if (rc) return rc;
  bumbar_options opt;
  if (opt_in)
    opt = *opt_in;
  else
    bumbar_default_options(&opt);
  if (!N_k || !f_k || !workspace) return fail(ctx, BUMBAR_EINVAL, "NULL argument");
  if (model != BUMBAR_MODEL_NONE && !coef) return fail(ctx, BUMBAR_EINVAL, "model needs coef");
  if ((opt.binning || otf) && !xi_in) return fail(ctx, BUMBAR_EINVAL, "xi is NULL");
  opt.xi_dtype = xi_dtype;  // the call's type decides the plan
  Plan plan;
  {
    std::string why;
    rc = make_plan(opt, otf, u_dtype, K, N, opt.binning || otf ? d : 0, model, &plan, &why);
    if (rc) return fail(ctx, rc, "%s", why.c_str());
  }
  const int rep = plan.rep;
  const bool mixed = plan.mixed;
  // counts: host copy for validation
  std::vector<int64_t> nk(K);
  rc = read_bytes(ctx, N_k, nk.data(), sizeof(int64_t) * K);
  if (rc) return rc;
  int64_t tot = 0;
  for (int k = 0; k < K; ++k) {
    if (nk[k] < 0) return fail(ctx, BUMBAR_EINVAL, "negative N_k");
    tot += nk[k];
  }
  if (tot != N) return fail(ctx, BUMBAR_EINVAL, "sum of N_k (%lld) != N (%lld)", (long long)tot,
                            (long long)N);
  // the plan's buffers, in the order of the workspace queries
  Arena ar{reinterpret_cast<char*>(workspace), ws_bytes};
  PlanBufs pb;
  carve_plan(ar, plan, ctx->num_cus, &pb);
  if (ar.overflow)
    return fail(ctx, BUMBAR_ENOMEM, "workspace too small (%zu bytes, need %zu)", ws_bytes, ar.off);
  UnbinnedBufs& B = pb.B;
  BinnedBufs& BB = pb.BB;
  MixedBufs& X = pb.X;
  OtfBufs& O = pb.O;
  if (opt.binning) BB.otf = rep == BUMBAR_REPRESENT_CENTRE;
  // every buffer a planned path launches with must have been carved
  if ((plan.x_packed && !X.r) || (plan.copy && !pb.copy) || (plan.o_bufs && !O.cf64) ||
      (plan.fp32_binned && !BB.cenf[0]) || (plan.xi_wide && !pb.xi64) || (plan.p16 && !pb.p16))
    return fail(ctx, BUMBAR_EINVAL, "internal: a planned buffer was not carved");
  // the coordinates every kernel reads: the caller's FP64 array, or FP32
  // coordinates widened (exactly) into the workspace
  const double* xi = reinterpret_cast<const double*>(xi_in);
  if (plan.xi_wide) {
    const hipError_t ew =
        launch_widen_f32(ctx->stream, reinterpret_cast<const float*>(xi_in), N * d, pb.xi64);
    if (ew != hipSuccess) return hip_fail(ctx, ew, "widen coordinates");
    xi = pb.xi64;
  }
  bumbar_stats local{};
  bumbar_stats* st = stats ? stats : &local;
  bumbar_check* chk = st->checks;
  int chk_cap = st->checks_capacity;
  // a trace file needs the schedule even if the caller keeps none: then the
  // solve records it in its own buffer, and on every return path the
  // caller's buffer gets back its place in the statistics, with what fits
  struct TraceChecks {
    bumbar_stats* st;
    bumbar_check* caller;
    int cap;
    std::vector<bumbar_check> buf;
    ~TraceChecks() {
      if (buf.empty()) return;
      const int64_t n = std::min<int64_t>(st->n_checks, caller ? cap : 0);
      if (n > 0) std::memcpy(caller, buf.data(), sizeof(bumbar_check) * (size_t)n);
      st->checks = caller;
      st->checks_capacity = cap;
    }
  } trace_checks{st, chk, chk_cap, {}};
  if (opt.trace_path && (!chk || chk_cap < kTraceChecks)) {
    trace_checks.buf.resize(kTraceChecks);
    chk = trace_checks.buf.data();
    chk_cap = kTraceChecks;
  }
  std::memset(st, 0, sizeof(*st));
  st->checks = chk;
  st->checks_capacity = chk_cap;
  hipStream_t s = ctx->stream;
  Mat M = input_mat(u_kn, u_dtype, N);
  M.p16 = pb.p16;    // the FP16 copy of P for the Newton Hessian (K > 256), or null
  SepGrid sep_grid;  // product-grid factors of the model, when they apply
  hipError_t e;
  if (otf) {
    M.kind = 4;
    M.otf.xi = xi;
    M.otf.xf = O.xf;
    M.otf.coef = coef;
    M.otf.d = d;
    M.otf.model = model;
    M.otf.cf32 = O.cf32;
    M.otf.cf64 = O.cf64;
    if (mixed) {
      e = launch_pack_coords(s, N * d, xi, O.xf);
      if (e != hipSuccess) return hip_fail(ctx, e, "pack coordinates");
    }
    bool on = false;
    rc = sep_setup(ctx, K, d, model, coef, O, &sep_grid, &on);
    if (rc) return rc;
    if (on) M.otf.sep = &sep_grid;
  }
  if (plan.copy) {
    // the sample-major copy every unbinned sweep of this solve reads; a NaN
    // in u is caught here once, not in every sweep
    e = hipMemsetAsync(B.nan_flag, 0, sizeof(unsigned), s);
    if (e == hipSuccess) e = launch_smaj_copy(s, u_kn, plan.copy_f32, N, K, N, pb.copy, B.nan_flag);
    if (e != hipSuccess) return hip_fail(ctx, e, "sample-major copy");
    unsigned nan_seen = 0;
    rc = read_bytes(ctx, B.nan_flag, &nan_seen, sizeof(unsigned));
    if (rc) return rc;
    if (nan_seen) return fail(ctx, BUMBAR_EINVAL, "u_kn holds a NaN");
    M.ut = pb.copy;
    M.ut_f32 = plan.copy_f32;
    M.ut_checked = true;
  }
  SweepCounters cnt;
  ctx->profiling = opt.profile != 0;
  ctx->events_used = 0;
  // kept states of the reduced Newton system (all sampled states but the
  // first), uploaded once for the blocked solve of large systems
  std::vector<int> kept;
  for (int k = 0, first = 1; k < K; ++k)
    if (nk[k] > 0) {
      if (!first) kept.push_back(k);
      first = 0;
    }
  if ((int)kept.size() > newton_lds_max_m()) {
    e = hipMemcpyAsync(B.idx, kept.data(), sizeof(int) * kept.size(), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "upload idx");
    B.m_red = (int)kept.size();
  }
  if (f_init && !opt.binning)
    e = hipMemcpyAsync(B.f, f_init, sizeof(double) * K, hipMemcpyDeviceToDevice, s);
  else
    e = hipMemsetAsync(B.f, 0, sizeof(double) * K, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "init f");

  int stage_rc = BUMBAR_OK;
  if (opt.binning) {
    // bin-centre representatives: the FP64 model evaluated in the binned sweeps
    Mat Mc;
    Mc.kind = 4;
    Mc.otf.xi = xi;
    Mc.otf.xf = O.xf;
    Mc.otf.coef = coef;
    Mc.otf.d = d;
    Mc.otf.model = model;
    Mc.otf.cf32 = O.cf32;
    Mc.otf.cf64 = O.cf64;
    Mc.otf.sep = M.otf.sep;
    // MEAN ignores a given model: the representatives are the bin means of u
    const int rep_model = rep == BUMBAR_REPRESENT_MEAN ? BUMBAR_MODEL_NONE : model;
    // In mixed precision with K > 256 and bin-centre representatives (where a
    // binned step is a compute-bound model sweep over K x P, not a few
    // launches) the binned steps first run on the FP32 model sweep. That stage only provides the
    // Newton start, but FP32 rounding of large energies can keep its
    // relative-step tests from passing: if it has not converged within
    // kFp32BinnedSteps steps it is rerun in FP64 from the start. For smaller K
    // the FP32 noise costs more iterations than it saves per step.
    constexpr int64_t kFp32BinnedSteps = 4000;
    // (a product grid of windows steps faster on the factored FP64 sweep)
    const bool try32 = plan.fp32_binned && !M.otf.sep;
    if (try32) {
      bumbar_options o32 = opt;
      o32.max_iter = std::min<int64_t>(opt.max_iter, kFp32BinnedSteps);
      stage_rc = binned_stage(ctx, B, BB, nullptr, N_k, nk.data(), xi, d, rep_model, coef, o32, st,
                              &cnt, &Mc, true);
      if (stage_rc != BUMBAR_OK && stage_rc != BUMBAR_ENOTCONV) return stage_rc;
      if (stage_rc == BUMBAR_ENOTCONV && o32.max_iter < opt.max_iter) {
        e = hipMemsetAsync(B.f, 0, sizeof(double) * K, s);  // the binned stage starts at f = 0
        if (e != hipSuccess) return hip_fail(ctx, e, "init f");
        stage_rc = binned_stage(ctx, B, BB, nullptr, N_k, nk.data(), xi, d, rep_model, coef, opt,
                                st, &cnt, &Mc, false);
      }
    } else {
      stage_rc = binned_stage(ctx, B, BB, reinterpret_cast<const double*>(u_kn), N_k, nk.data(),
                              xi, d, rep_model, coef, opt, st, &cnt, BB.otf ? &Mc : nullptr);
    }
    if (stage_rc != BUMBAR_OK && stage_rc != BUMBAR_ENOTCONV) return stage_rc;
  } else if (opt.finisher == BUMBAR_FINISH_NEWTON) {
    const double t0 = now_ms();
    int64_t it = 0;
    double last = 0;
    stage_rc = sci_until(ctx, B, M, N_k, opt.sci_switch, opt.max_iter, &it, &cnt, &last);
    if (stage_rc != BUMBAR_OK && stage_rc != BUMBAR_ENOTCONV) return stage_rc;
    st->phase1_iters = it;
    st->time_binned_ms = now_ms() - t0;
  }
  const double t1 = now_ms();
  int fin_rc = BUMBAR_OK;
  int64_t steps64 = 0;  // Newton steps on M itself (after any packed stage)
  // Newton on a product grid in mixed precision: the factored FP64 sweeps
  // (cheaper than the direct FP32 ones) with the Hessian from the FP32 model
  Mat Mfin = M;
  if (mixed && otf && M.otf.sep) Mfin.hess_kind = 3;
  // stored u: the planned Newton Hessian source (it only shapes the steps;
  // the FP64 sweeps decide the fixed point)
  if (!otf) Mfin.hess_kind = plan.hess_kind;
  if (stage_rc == BUMBAR_OK) {
    if (opt.finisher == BUMBAR_FINISH_NEWTON) {
      if (mixed && otf && !M.otf.sep) {
        // Newton on the FP32 model sweeps to mixed_tol, then FP64 refinement
        // (on a product grid the FP64 Newton below takes all the steps)
        Mat R = M;
        R.kind = 3;
        const double mtol = opt.mixed_tol > opt.tol ? opt.mixed_tol : opt.tol;
        const int64_t before = st->finisher_steps;
        int mrc = newton_finish(ctx, B, R, N_k, mtol, opt.max_newton, st, &cnt, &st->final_step,
                                &st->grad_norm);
        if (mrc != BUMBAR_OK && mrc != BUMBAR_ENOTCONV) return mrc;
        st->mixed_steps = st->finisher_steps - before;
      } else if (mixed && (plan.stage32 == BUMBAR_STAGE32_SAMPLE_MAJOR ||
                           plan.stage32 == BUMBAR_STAGE32_STORED)) {
        // Newton on FP32-exponential sweeps of the sample-major copy (or of
        // the stored FP32 u, K <= 256) to mixed_tol, then FP64 refinement on
        // the same data to tol
        Mat R = M;
        R.kind = 7;
        R.hess_kind = plan.hess_kind32;
        const double mtol = opt.mixed_tol > opt.tol ? opt.mixed_tol : opt.tol;
        const int64_t before = st->finisher_steps;
        int mrc = newton_finish(ctx, B, R, N_k, mtol, opt.max_newton, st, &cnt, &st->final_step,
                                &st->grad_norm);
        if (mrc != BUMBAR_OK && mrc != BUMBAR_ENOTCONV) return mrc;
        st->mixed_steps = st->finisher_steps - before;
      } else if (mixed && plan.stage32 == BUMBAR_STAGE32_PACKED) {
        // pack at the current f, Newton on the FP32 matrix to mixed_tol, then
        // FP64 refinement on u to tol
        e = launch_prepare_consts(s, K, N_k, B.f, B.cst, B.gk, B.lnNp);
        if (e == hipSuccess) e = launch_pack_f32(s, u_kn, u_dtype == BUMBAR_F32, N, K, N, B.cst,
                                                 X.r, N, X.m0);
        if (e == hipSuccess)
          e = hipMemcpyAsync(X.f0, B.f, sizeof(double) * K, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "pack");
        Mat R;
        R.u = X.r;
        R.kind = 2;
        R.ld = N;
        R.m0 = X.m0;
        R.f0 = X.f0;
        const double mtol = opt.mixed_tol > opt.tol ? opt.mixed_tol : opt.tol;
        const int64_t before = st->finisher_steps;
        int mrc = newton_finish(ctx, B, R, N_k, mtol, opt.max_newton, st, &cnt, &st->final_step,
                                &st->grad_norm);
        if (mrc != BUMBAR_OK && mrc != BUMBAR_ENOTCONV) return mrc;
        st->mixed_steps = st->finisher_steps - before;
      }
      const int64_t before64 = st->finisher_steps;
      fin_rc = newton_finish(ctx, B, Mfin, N_k, opt.tol, opt.max_newton, st, &cnt,
                             &st->final_step, &st->grad_norm);
      steps64 = st->finisher_steps - before64;
    } else {
      int64_t it = 0;
      const int64_t left = std::max<int64_t>(0, opt.max_iter - st->phase1_iters - st->phase2_iters);
      fin_rc = sci_until(ctx, B, M, N_k, opt.tol, left, &it, &cnt, &st->final_step);
      st->finisher_steps = it;
    }
    if (fin_rc != BUMBAR_OK && fin_rc != BUMBAR_ENOTCONV) return fin_rc;
  }
  st->time_final_ms = now_ms() - t1;
  // outputs: ln D at the final f, weights, f. After Newton steps the last
  // sweep was at the final f up to the gauge shift (which leaves the
  // gradient unchanged), so a new sweep is needed only for ln D and W.
  const bool newton_done = stage_rc == BUMBAR_OK && opt.finisher == BUMBAR_FINISH_NEWTON &&
                           steps64 > 0;
  if (!newton_done || log_D_n || W_nk) {
    SweepScalars sc{};
    rc = sweep_at(ctx, B, M, N, nullptr, N_k, B.f, B.f_new, B.logD, B.lnS, B.S, &sc, false, &cnt);
    if (rc) return rc;
    st->grad_norm = sc.grad_norm;
  }
  e = hipMemcpyAsync(f_k, B.f, sizeof(double) * K, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && log_D_n)
    e = hipMemcpyAsync(log_D_n, B.logD, sizeof(double) * N, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && W_nk)
    e = otf ? launch_weights_otf(s, M.otf, K, N, B.f, B.logD, W_nk)
            : launch_weights(s, u_kn, u_dtype == BUMBAR_F32, N, K, N, B.f, B.logD, W_nk);
  if (e == hipSuccess) e = ctx_wait(ctx, s);
  if (e != hipSuccess) return hip_fail(ctx, e, "outputs");
  st->unbinned_sweeps = cnt.fast + cnt.robust;
  st->robust_sweeps = cnt.robust;
  st->grid_sweeps = cnt.grid;
  if (ctx->profiling) st->sweep_kernel_ms = collect_event_ms(ctx, &st->sweep_kernel_launches);
  ctx->profiling = false;
  if (opt.trace_path) {
    rc = write_trace(ctx, opt.trace_path, K, N, *st);
    if (rc) return rc;
  }
  if (stage_rc == BUMBAR_ENOTCONV || fin_rc == BUMBAR_ENOTCONV)
    return fail(ctx, BUMBAR_ENOTCONV, "iteration cap reached before convergence");
  return BUMBAR_OK;
}

}  // extern "C"
