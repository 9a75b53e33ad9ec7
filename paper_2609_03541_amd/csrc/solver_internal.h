// Host-side helpers shared by solver.cpp (unbinned sweeps, Newton finisher,
// C ABI) and algo.cpp (binning and Algorithm 1).
#pragma once

#include <cstdarg>
#include <cstdint>
#include <string>

#include "bumbar_impl.h"

namespace bumbar {

int fail(bumbar_ctx* ctx, int code, const char* fmt, ...);
int hip_fail(bumbar_ctx* ctx, hipError_t e, const char* where);
double now_ms();
int read_bytes(bumbar_ctx* ctx, const void* dev, void* host, size_t bytes);
// Waits for the work queued on s: hipStreamSynchronize, or, for a solve
// running as a fiber of a caller-driven server, yields to the server while
// the stream is busy.
hipError_t ctx_wait(bumbar_ctx* ctx, hipStream_t s);
std::pair<hipEvent_t, hipEvent_t>* next_event_pair(bumbar_ctx* ctx);

// Binned SCI steps queued between two host readbacks.
constexpr int kHistSteps = 32;

struct SweepCounters {
  int64_t fast = 0;
  int64_t robust = 0;
  int64_t grid = 0;  // FP64 model sweeps completed on the product-grid passes
};

// The matrix a sweep reads: FP64 u, FP32 u (widened to FP64 arithmetic), the
// packed mixed-precision matrix r_kn = fp32(c0_k - u_kn - m0_n) taken at the
// reference point f0 (FP32 arithmetic inside the sweep), or u from the bias
// model evaluated inside the kernels (FP32 or FP64 arithmetic).
struct Mat {
  const void* u = nullptr;
  int kind = 0;  // 0: FP64, 1: FP32, 2: packed, 3: model FP32, 4: model FP64,
                 // 7: FP32 arithmetic over the sample-major copy (ut)
  int64_t ld = 0;
  const double* m0 = nullptr;  // kind 2: per-column shift (N)
  const double* f0 = nullptr;  // kind 2: reference point (K)
  OtfModel otf;                // kinds 3 and 4
  int hess_kind = -1;          // kind the Newton Hessian reads (-1: kind; 5: FP64 u
                               // on the FP16 matrix cores; 6: FP64 u, FP32 exponentials)
  const void* ut = nullptr;    // the sample-major copy the sweeps read (kinds 0, 1, 7), or null
  bool ut_f32 = false;         // its element type
  bool ut_checked = false;     // made by the solve (NaN checked once by the copy kernel)
  void* p16 = nullptr;         // FP16 copy of P for the FP16-core Hessian (K > 256), or null
};

// Coordinates in FP32 and the per-sweep model coefficients of the
// on-the-fly kinds (carved whenever coordinates are given).
struct OtfBufs {
  float* xf = nullptr;
  float* cf32 = nullptr;
  double* cf64 = nullptr;
  int* sep_i = nullptr;     // d = 2: product-grid maps and cells (SepGrid)
  double* sep_d = nullptr;  // d = 2: product-grid factors, C and cmax
  void carve(Arena& ar, int K, int64_t N, int d) {
    xf = ar.take<float>((size_t)N * d);
    cf32 = ar.take<float>(otf_coef_floats(K, d));
    cf64 = ar.take<double>(otf_coef_floats(K, d));
    if (d == 2) {
      sep_i = ar.take<int>(sep_int_count(K));
      sep_d = ar.take<double>(sep_double_count());
    }
  }
};

// Device buffers for sweeps and the Newton finisher of one K x N problem.
struct UnbinnedBufs {
  int K = 0;
  int64_t N = 0;
  double *cst = nullptr, *gk = nullptr, *lnNp = nullptr;
  double *f = nullptr, *f_new = nullptr, *f_trial = nullptr, *dir = nullptr;
  double* f_sweep = nullptr;  // the point of the sweep whose ln D the Hessian uses
  double *lnS = nullptr, *S = nullptr, *lnS_t = nullptr, *S_t = nullptr;
  double *logD = nullptr, *logD_t = nullptr;
  int nparts_cap = 0;
  double *part = nullptr, *partS = nullptr, *part_obj = nullptr;
  unsigned* part_flags = nullptr;
  SweepScalars* scal = nullptr;
  SweepScalars* scal_hist = nullptr;  // kHistSteps per-step scalars (binned batches)
  double* f_hist = nullptr;           // kHistSteps x K iterates (binned batches)
  double* misc = nullptr;
  int* ok = nullptr;
  unsigned* nan_flag = nullptr;  // set by the sample-major copy when u holds a NaN
  int* idx = nullptr;
  double *A = nullptr, *H = nullptr, *hess_parts = nullptr;
  double* dk = nullptr;  // f - f0 for the packed matrix
  int hess_chunks = 1;
  bool H_valid = false;  // H holds a Hessian usable for chord steps
  int m_red = -1;        // reduced Newton size when idx was uploaded by the host, else -1
  void carve(Arena& ar, int K, int64_t N, int num_cus);
};

// Extra device buffers of the packed mixed-precision stage (K <= 256).
struct MixedBufs {
  float* r = nullptr;     // K x N packed matrix
  double* m0 = nullptr;   // N
  double* f0 = nullptr;   // K
  void carve(Arena& ar, int K, int64_t N) {
    r = ar.take<float>((size_t)K * (size_t)N);
    m0 = ar.take<double>(N);
    f0 = ar.take<double>(K);
  }
};

// What bumbar_solve runs and which workspace buffers it carves, decided on
// the host from the call's shapes and options alone (plan.cpp). The solve,
// the workspace queries and bumbar_plan_solve share it, so the buffers a
// path launches with are exactly the ones carved for it.
struct Plan {
  bool otf = false;        // energies from the model (u_kn = NULL)
  int u_dtype = BUMBAR_F64;
  int K = 0;
  int64_t N = 0;
  int d = 0;
  bool binning = false;
  int rep = 0;             // resolved representative (binning only)
  bool mixed = false;      // an FP32 Newton stage runs before the FP64 one
  int sweep = BUMBAR_SWEEP_REGISTER;
  int stage32 = BUMBAR_STAGE32_NONE;
  bool fp32_binned = false;  // binned steps first on the FP32 model sweep
  bool copy = false;         // sample-major copy of u in the workspace
  bool copy_f32 = false;     // its element type
  bool xi_wide = false;      // FP32 coordinates widened to FP64 in the workspace
  bool p16 = false;          // FP16 copy of P (K x p16_samples(K, N)) for the Newton Hessian
  // carve flags
  bool bb_ubar = false, bb_cen = false, bb_cen_f32 = false;
  int64_t bb_otf_cap = 0;
  bool x_packed = false, o_bufs = false;
  int hess_kind = -1;      // Newton Hessian source of the FP64 stage (-1: the sweep's kind)
  int hess_kind32 = -1;    // and of the FP32 stage
  size_t copy_bytes() const;
};

// Fills *p; returns BUMBAR_OK or BUMBAR_EINVAL with the reason in *msg.
int make_plan(const bumbar_options& opt, bool otf, int u_dtype, int K, int64_t N, int d,
              int model, Plan* p, std::string* msg);

// One sweep of M at f. With a packed matrix a flagged sweep (weights outside
// the FP32 range) is reported through sc->flags and not redone.
int sweep_at(bumbar_ctx* ctx, const UnbinnedBufs& B, const Mat& M, int64_t N, const double* h,
             const int64_t* Nk, const double* f, double* f_out, double* logD_out,
             double* lnS_out, double* S_out, SweepScalars* sc, bool force_robust,
             SweepCounters* cnt);

// Queues one sweep without reading anything back. consts_ready: B.cst / B.gk
// / B.lnNp already hold the constants at f (skip their rebuild); cst_next:
// where the finaliser writes the constants at f_out for a following step
// (may be B.cst itself), or nullptr.
int sweep_queue(bumbar_ctx* ctx, const UnbinnedBufs& B, const Mat& M, int64_t N, const double* h,
                const int64_t* Nk, const double* f, double* f_out, double* logD_out,
                double* lnS_out, double* S_out, SweepScalars* dev_scal,
                bool consts_ready = false, double* cst_next = nullptr);

int newton_finish(bumbar_ctx* ctx, UnbinnedBufs& B, const Mat& M, const int64_t* Nk, double tol,
                  int max_steps, bumbar_stats* st, SweepCounters* cnt, double* final_step,
                  double* final_gnorm);

// Resolves this device's address of the fixed scratch array behind
// bumbar_sweep_static into ctx->static_scratch (ctx->device current).
int static_scratch_init(bumbar_ctx* ctx);

int sci_until(bumbar_ctx* ctx, UnbinnedBufs& B, const Mat& M, const int64_t* Nk, double until,
              int64_t max_steps, int64_t* steps_out, SweepCounters* cnt, double* last_step);

// ---- binning ---------------------------------------------------------------

struct Level {
  int64_t n = 0;   // nominal target
  uint64_t m = 0;  // width in quanta
  int64_t P = 0;   // nonempty bins
  double* ubar = nullptr;  // K x P (row stride P), or P x Kp (smaj); stored representatives
  bool smaj = false;       // ubar in the sample-major layout (256 < K <= 1024)
  double* cen = nullptr;   // P x d bin centres; representatives from the model
  float* cenf = nullptr;   // the same centres in FP32 (mixed precision), or null
  double* h = nullptr;     // P multiplicities (as double)
};

struct BinnedBufs {
  int d = 0;
  int64_t N = 0;
  uint32_t* q = nullptr;         // N x d quantised coordinates
  double* lo = nullptr;          // d
  double* scale = nullptr;       // d
  double* mm = nullptr;          // 2 d min / max
  uint64_t* keys = nullptr;      // N cell ids (unsorted)
  uint64_t* keys_sorted = nullptr;
  uint32_t* iota = nullptr;      // N: 0..N-1
  uint32_t* perm = nullptr;      // N: sample index of each sorted position
  uint32_t* q1_sorted = nullptr; // 1-D: sorted q (sorted once)
  uint32_t* perm1 = nullptr;     // 1-D: permutation of the one-time sort
  uint64_t* q2_sorted = nullptr; // 2-D: the pairs sorted by (q_y, q_x) (sorted once)
  int32_t* bin_of_pos = nullptr; // N: bin index of each sorted position
  int64_t* start = nullptr;      // N + 1: first sorted position of each bin
  uint64_t* cells = nullptr;     // N: cell id of each bin
  int64_t* counts = nullptr;     // reduction scratch
  int64_t g1 = -1;               // g(1), the distinct quantised points (once per solve)
  void* sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
  bool otf = false;                      // representatives from the model in the kernels
  // K x N each (worst case P = N) in stored mode; on the fly, K x ubar_cap
  // each: levels with P <= ubar_cap get their centre representatives
  // materialised (one model evaluation per level) and step like stored ones
  double* ubar[2] = {nullptr, nullptr};
  int64_t ubar_cap = 0;
  int ubar_row = 0;  // values per bin of a materialised level: K, or Kp sample-major
  double* cen[2] = {nullptr, nullptr};   // N x d each (worst case P = N); otf mode
  float* cenf[2] = {nullptr, nullptr};   // FP32 copies of cen (mixed precision)
  double* h[2] = {nullptr, nullptr};     // N each
  double* logD_lvl = nullptr;            // N
  double* coop = nullptr;                // scratch of the cooperative batches (256 < K <= 1024)
  double *f_n = nullptr, *f_x = nullptr; // K
  // ubar_bufs: K x N representative buffers (MEAN); cen_bufs: N x d centres
  // (CENTRE), cen_f32 also their FP32 copies; otf_cap > 0: K x otf_cap
  // representative buffers for the small levels of an on-the-fly stage. otf
  // is set by the caller to the representative in use.
  void carve(Arena& ar, int K, int64_t N, int d, int num_cus, bool ubar_bufs, bool cen_bufs,
             bool cen_f32 = false, int64_t otf_cap = 0);
};

void binned_carve_size(Arena& ar, int K, int64_t N, int d, int num_cus, bool ubar_bufs,
                       bool cen_bufs, bool cen_f32 = false, int64_t otf_cap = 0);

// On the fly with K states: the largest level (in bins) whose centre
// representatives are materialised, or 0 (K beyond the register-tiled sweep).
int64_t otf_ubar_cap(int K, int64_t N);

// otf_base: nullptr for stored representatives, else the FP64 model matrix
// (kind 4) whose coordinates the stage replaces by the bin centres. With
// fp32_steps and FP32 centres (BinnedBufs::cenf) the batched steps run the
// FP32 model sweep and only steps that need a fallback run in FP64.
int binned_stage(bumbar_ctx* ctx, UnbinnedBufs& B, BinnedBufs& BB, const double* u,
                 const int64_t* Nk_dev, const int64_t* Nk_host, const double* xi, int d,
                 int model, const double* coef, const bumbar_options& opt, bumbar_stats* st,
                 SweepCounters* cnt, const Mat* otf_base, bool fp32_steps = false);

// Binning primitives (binning.hip).
size_t sort_temp_bytes(int64_t N);
hipError_t launch_minmax(hipStream_t s, const double* xi, int64_t N, int d, double* mm,
                         int64_t* scratch);
hipError_t launch_quantize(hipStream_t s, const double* xi, int64_t N, int d, const double* mm,
                           double* lo, double* scale, uint32_t* q, unsigned* bad);
hipError_t launch_sort_1d(hipStream_t s, const uint32_t* q, int64_t N, uint32_t* iota,
                          uint32_t* q_sorted, uint32_t* perm, void* tmp, size_t tmp_bytes);
// g(m) for 1-D sorted coordinates or 2-D (sorts the cell ids of this m); result
// in counts[0] after the call.
hipError_t launch_count_1d(hipStream_t s, const uint32_t* q_sorted, int64_t N, uint64_t m,
                           int64_t* counts);
// The 1-D width search on the device: the bisection for max{m : g(m) >= n}
// on [1, 2^32] with the midpoints of `levels` levels of the tree counted per
// pass (count kernel) and the path walked between passes (one-thread walk
// kernel), so the host reads back only the result. init starts a search;
// `passes` count + walk pairs are queued (passes after the end do nothing).
// Result: lo (= m), glo (= g(m)), done.
struct WidthSearch1D {
  uint64_t lo, hi;
  int64_t glo, n;
  int levels, M, done, first;
  uint64_t ms[2 * 64];              // (m, ceil(2^64 / m)) pairs of this pass
  unsigned long long counts[64];    // g of each probe
};
hipError_t launch_width_search_1d(hipStream_t s, const uint32_t* q_sorted, int64_t N,
                                  int64_t n, int levels, int passes, bool init,
                                  WidthSearch1D* w);
// The 2-D width search on the device: the same bisection, one probe per
// pass, each probe an occupancy bitmap of its grid (at most 64 N cells, in
// the N x 8-byte buffer `bitmap`); the walk ends the search (done) or hands
// it back (host = 1) when the next grid does not fit. init starts it from
// lo = 1 with g(1) = g1 given; `passes` passes are queued.
struct WidthSearch2D {
  uint64_t lo, hi;
  int64_t glo, n;
  uint64_t m, magic, ncx, cap_cells;
  int64_t nw;
  unsigned long long count;
  int done, host;
};
// Probes over q2_sorted (the 2-D coordinates sorted by launch_sort_2d).
hipError_t launch_width_search_2d(hipStream_t s, const uint64_t* q2_sorted, int64_t N, int64_t n,
                                  int64_t g1, int passes, bool init, uint64_t* bitmap,
                                  WidthSearch2D* w);
// q2_sorted = the N quantised pairs as keys q_y 2^32 + q_x in ascending order
// (keys: N entries of scratch); counts[0] = their distinct values, g(1).
hipError_t launch_sort_2d(hipStream_t s, const uint32_t* q, int64_t N, uint64_t* keys,
                          uint64_t* q2_sorted, void* tmp, size_t tmp_bytes);
hipError_t launch_count_sorted_2d(hipStream_t s, const uint64_t* q2_sorted, int64_t N,
                                  int64_t* counts);
hipError_t launch_count_2d(hipStream_t s, const uint32_t* q, int64_t N, uint64_t m,
                           uint64_t* keys, uint64_t* keys_sorted, void* tmp, size_t tmp_bytes,
                           int64_t* counts);
// Histogram at width m: bins in ascending cell order. On return counts[0] = P
// (device); cells, start (P + 1 entries), bin_of_pos, perm filled.
hipError_t launch_histogram(hipStream_t s, const uint32_t* q, int64_t N, int d, uint64_t m,
                            const uint32_t* q1_sorted, const uint32_t* perm1, uint32_t* iota,
                            uint64_t* keys, uint64_t* keys_sorted, uint32_t* perm,
                            int32_t* bin_of_pos, int64_t* start, uint64_t* cells, void* tmp,
                            size_t tmp_bytes, int64_t* counts);
hipError_t launch_represent(hipStream_t s, int K, int64_t N, int d, int model, const double* coef,
                            const double* lo, const double* scale, uint64_t m, int64_t P,
                            const uint64_t* cells, const int64_t* start, const uint32_t* perm,
                            const double* u, double* ubar, double* h);
hipError_t launch_centres(hipStream_t s, int d, const double* lo, const double* scale, uint64_t m,
                          int64_t P, const uint64_t* cells, const int64_t* start, double* cen,
                          double* h);
// out (P x Kp) = model_k(cen_p), +inf past K: bin-centre representatives in
// the sample-major layout.
hipError_t launch_represent_smaj(hipStream_t s, int K, int Kp, int d, int model,
                                 const double* coef, int64_t P, const double* cen, double* out);
hipError_t launch_sample_bin(hipStream_t s, int64_t N, const uint32_t* perm,
                             const int32_t* bin_of_pos, int32_t* sample_bin);
hipError_t launch_counts_from_start(hipStream_t s, int64_t P, const int64_t* start, int64_t* H);

// Carves the plan's buffers in a fixed order (the solve and the queries).
struct PlanBufs {
  UnbinnedBufs B;
  BinnedBufs BB;
  MixedBufs X;
  OtfBufs O;
  void* copy = nullptr;
  double* xi64 = nullptr;  // N x d widened coordinates (xi_wide)
  void* p16 = nullptr;     // K x p16_samples(K, N) halves (Plan::p16)
};
void carve_plan(Arena& ar, const Plan& p, int num_cus, PlanBufs* pb);

}  // namespace bumbar
