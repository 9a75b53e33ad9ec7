// Internal declarations of libbumbar (not installed; the public ABI is include/bumbar.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "bumbar.h"

namespace bumbar {

// Scalars produced by the sweep finaliser (device memory, read back on demand).
struct SweepScalars {
  double max_df;    // max_k |f_new_k - f_k|
  double rel_step;  // Eq. (2), gauge state excluded
  double objective; // sum_n h_n ln D_n - sum_k N_k f_k
  double grad_norm; // || S - N ||_2 over sampled states
  double min_S;     // min over sampled states of S_k
  unsigned flags;   // bit 0: column denominator underflow / non-finite;
                    // bit 1: state sum underflow / non-finite (robust path needed)
  unsigned pad;
};

enum : unsigned { FLAG_COL = 1u, FLAG_STATE = 2u, FLAG_NAN = 4u };

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures, which is how bumbar_query_workspace sizes the same sequence.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t off = 0;
  bool overflow = false;
  template <typename T>
  T* take(size_t count) {
    size_t bytes = count * sizeof(T);
    size_t start = (off + 255) & ~size_t(255);
    off = start + bytes;
    if (base == nullptr) return nullptr;
    if (off > cap) {
      overflow = true;
      return nullptr;
    }
    return reinterpret_cast<T*>(base + start);
  }
};

// ---- sweep kernels (sweep.hip) ------------------------------------------

// Per-problem constants staged on the device for the sweeps.
struct SweepConsts {
  const double* cst;  // K: ln N'_k + f_k (N'_k = N_k if N_k > 0 else 1)
  const double* gk;   // K: 1 if N_k > 0 else 0
};

int sweep_max_grid(int num_cus);                // upper bound for workspace sizing
int robust_chunks(int64_t N);                   // column chunks of the robust pass

// Fast single-pass sweep. Writes per-block partial state sums (grid x K),
// per-block objective partials and flags. h (per-column multiplicity) may be
// null; logD may be null. Returns 0 or a hipError_t value.
// The grid (persistent, occupancy-sized) is returned in *grid_out. u is FP64,
// or FP32 (f32) widened exactly on load; the arithmetic is FP64, except that
// f32_arith (FP32 storage only: the FP32 stage of mixed precision) takes the
// exponentials of the FP64-shifted exponents in FP32 (hardware exp2).
hipError_t launch_sweep_fast(hipStream_t s, const void* u, bool f32, bool f32_arith, int64_t ld,
                             int K, int64_t N, const double* cst, const double* gk,
                             const double* h, double* logD, double* part, double* part_obj,
                             unsigned* part_flags, int num_cus, int* grid_out);
bool sweep_fast_supported(int K);

// Robust two-pass sweep: exact column max, then per-state online log-sum-exp.
// u is FP64, or FP32 when f32 (widened on load); state-major with row stride
// ld, or (sample_major) the sample-major copy with rows of ld values.
hipError_t launch_sweep_robust(hipStream_t s, const void* u, bool f32, int64_t ld, int K, int64_t N,
                               const double* cst, const double* gk, const double* h,
                               double* logD, double* partM, double* partS, double* part_obj,
                               unsigned* part_flags, int chunks, bool sample_major = false);

// Sample-major copy of u for 256 < K <= 1024 (sweep_smaj.hip): N rows of
// Kp = smaj_row(K) = 64 J values (J in {5, 6, 8, 10, 12, 14, 16}, the smallest
// with K <= 64 J), states past K = +inf, so that a
// sample is one contiguous row; smaj_elems = N Kp. launch_smaj_copy sets
// *nan_flag (if given; the caller zeroes it) when u holds a NaN.
// launch_sweep_smaj: the single-pass sweep over the copy, one wavefront per
// sample pair, in FP64 arithmetic (FP64 copy, or FP32 copy widened) or, with
// f32_arith, FP32 exponentials (mixed precision). nan_check: test every
// element for NaN (a copy the caller made); the solve's own copy was checked
// when it was made (f32_arith requires that).
int smaj_row(int K);
size_t smaj_elems(int K, int64_t N);
bool sweep_smaj_supported(int K);
hipError_t launch_smaj_copy(hipStream_t s, const void* u, bool f32, int64_t ld, int K, int64_t N,
                            void* ut, unsigned* nan_flag);
hipError_t launch_sweep_smaj(hipStream_t s, const void* ut, bool f32, bool f32_arith,
                             bool nan_check, int K, int64_t N, const double* cst,
                             const double* gk, const double* h, double* logD, double* part,
                             double* part_obj, unsigned* part_flags, int num_cus, int* grid_out);

// Finaliser. mode 0: partials are S' sums (fast path), partS a scratch of K
// doubles for their per-state sums (or null); mode 1: (M, S) pairs in
// (part, partS).
hipError_t launch_sweep_finalize(hipStream_t s, int mode, int K, int nparts, const double* part,
                                 double* partS, const double* part_obj,
                                 const unsigned* part_flags, const double* f, const double* lnNp,
                                 const int64_t* Nk, double* f_new, double* lnS, double* S_out,
                                 SweepScalars* out, double* cst_next = nullptr);

// T consecutive steps (sweep + finaliser, mode 0) of a stored K x P problem
// with column multiplicities h in one workgroup (sweep_small.hip): step i
// starts from f_in (i = 0) or f_hist row i - 1 and writes f_hist row i and
// scal[i]; ln D (P), ln S and S (K) of the last step; after the batch cst,
// gk and lnNp as launch_prepare_consts would leave them for the last f.
// small_batch_nc(K, P) is 0 where the batch kernel does not apply.
// Stable LSD radix sort (8-bit digits) of N < 2^32 keys over their low
// `bits` bits, with an optional 32-bit value per key (both value pointers
// set, or neither), and an inclusive scan of int32 (radix.hip). tmp:
// radix_temp_bytes(N) / scan_temp_bytes(N) bytes of device scratch. Inputs
// are not modified; outputs must not alias them.
size_t radix_temp_bytes(int64_t N);
size_t scan_temp_bytes(int64_t N);
hipError_t radix_sort_u32(hipStream_t s, const uint32_t* keys_in, uint32_t* keys_out,
                          const uint32_t* vals_in, uint32_t* vals_out, int64_t N, int bits,
                          void* tmp, size_t tmp_bytes);
hipError_t radix_sort_u64(hipStream_t s, const uint64_t* keys_in, uint64_t* keys_out,
                          const uint32_t* vals_in, uint32_t* vals_out, int64_t N, int bits,
                          void* tmp, size_t tmp_bytes);
hipError_t scan_inclusive_i32(hipStream_t s, const int32_t* in, int32_t* out, int64_t N,
                              void* tmp, size_t tmp_bytes);

int small_batch_nc(int K, int64_t P);
// The same batch on a level materialised in the sample-major layout (FP64,
// 256 < K <= 1024) as one cooperative launch (sweep_smaj.hip): grid
// barriers between each step's sweep, its per-state sums and its scalars.
// part: K x part_cap partials; wsc: smaj_batch_scratch(num_cus, T_max)
// doubles for batches of at most T_max steps. Also leaves ln S and S of
// the last step.
bool smaj_batch_supported(int K);
int64_t smaj_batch_scratch(int num_cus, int max_steps);
hipError_t launch_smaj_batch(hipStream_t s, const double* ut, int K, int64_t P, const double* h,
                             const int64_t* Nk, const double* f_in, int T, double* f_hist,
                             SweepScalars* scal, double* logD, double* lnS, double* S,
                             double* cst, double* gk, double* lnNp, double* part, int part_cap,
                             double* wsc, int wsc_steps, int num_cus);
// The arguments of one such batch (nc = small_batch_nc(K, P)).
struct SmallBatch {
  const double* u;
  int64_t ld;
  const double* h;
  const int64_t* Nk;
  const double* f_in;
  double* f_hist;
  SweepScalars* scal;
  double* logD;
  double* lnS;
  double* S;
  double* cst;
  double* gk;
  double* lnNp;
  int K, P, T, nc;
};
hipError_t launch_small_batch(hipStream_t s, const SmallBatch& a);
// Batches of several independent problems in one launch per column layout:
// a fixed grid of workgroups walks the items of its layout in the device
// work list (workgroup b takes items b, b + grid, ...); each item runs
// exactly the code of launch_small_batch, so its outputs are bitwise those
// of its own launch. Layout classes 0..3 are nc = 64, 128, 256, 512; the
// items of class c are items[first[c] .. first[c] + count[c]).
constexpr int kFusedGrid = 256;
struct SmallWorkHeader {
  int64_t count[4];
  int64_t first[4];
};
inline size_t small_work_bytes(int64_t count) {
  return sizeof(SmallWorkHeader) + (size_t)count * sizeof(SmallBatch);
}
int small_class(int nc);  // 0..3, -1 for an nc that is not a layout
// wl: device work list (header, then the items); a kernel of grid
// workgroups for each class whose bit is set in cls_mask.
hipError_t launch_small_fused(hipStream_t s, const SmallWorkHeader* wl, unsigned cls_mask,
                              int grid);

// cst_k = ln N'_k + f_k, gk, lnNp from N_k and f.
hipError_t launch_prepare_consts(hipStream_t s, int K, const int64_t* Nk, const double* f,
                                 double* cst, double* gk, double* lnNp);

// Small vector kernels.
hipError_t launch_axpy_to(hipStream_t s, int K, const double* f, double alpha, const double* d,
                          double* out);  // out = f + alpha d
hipError_t launch_fill_unsampled_gauge(hipStream_t s, int K, const int64_t* Nk, double* f,
                                       const double* lnS);
hipError_t launch_max_abs_diff(hipStream_t s, int K, const double* a, const double* b,
                               double* out);
hipError_t launch_weights(hipStream_t s, const void* u, bool f32, int64_t ld, int K, int64_t N,
                          const double* f, const double* logD, double* W);
hipError_t launch_reweight(hipStream_t s, int64_t N, const double* ut, const double* logD,
                           double* part, int nparts, double* p);
hipError_t launch_check_finite_f(hipStream_t s, int K, const double* f, unsigned* flag);

// ---- Hessian and linear algebra (hessian.hip, linalg.hip) ----------------
size_t hessian_partial_count(int K, int64_t N, int num_cus, int* chunks_out);
// Windows on a product grid (2-D harmonic): state k takes x-factor ix[k] and
// y-factor jy[k] among Ix and Jy distinct (kappa/2, centre) pairs, so the
// FP64 sweeps factor (sweep_otf.hip). Device arrays; cells c = i * Jy + j
// list their states in cstates[cstart[c] .. cstart[c + 1]).
constexpr int kSepMax = 64;  // factors per axis
struct SepGrid {
  int Ix = 0, Jy = 0, JM = 0;     // JM: Jy rounded up to a multiple of 8
  const double* fx = nullptr;     // kSepMax x 2: kappa_x / 2, centre x
  const double* fy = nullptr;     // kSepMax x 2
  const int* ix = nullptr;        // K
  const int* jy = nullptr;        // K
  const int* cstart = nullptr;    // Ix * Jy + 1
  const int* cstates = nullptr;   // K
  double* C = nullptr;            // Ix x JM, per sweep
  double* cmax = nullptr;         // 1, per sweep
};
size_t sep_int_count(int K);      // ints of a SepGrid's storage
size_t sep_double_count();        // doubles of a SepGrid's storage

// Reduced energies from the bias model, evaluated inside the kernels.
struct OtfModel {
  const double* xi = nullptr;    // N x d FP64 coordinates
  const float* xf = nullptr;     // N x d FP32 coordinates (FP32 kernels)
  const double* coef = nullptr;  // K x (1 + 2d) model coefficients
  int d = 0;
  int model = 0;                 // BUMBAR_MODEL_LINEAR or BUMBAR_MODEL_HARMONIC
  float* cf32 = nullptr;         // K x (2 + 2d) per-sweep FP32 coefficients
  double* cf64 = nullptr;        // K x (2 + 2d) per-sweep FP64 coefficients
  const SepGrid* sep = nullptr;  // host struct: product-grid factors, or null
};
size_t otf_coef_floats(int K, int d);  // entries of cf32 (and of cf64)
int otf_grid(int64_t N, int num_cus);
hipError_t launch_pack_coords(hipStream_t s, int64_t n, const double* xi, float* xf);
// Two-pass sweep with u from the model (FP32 or FP64 arithmetic) at the N
// points of m.xi / m.xf with multiplicities h (NULL: 1); also rebuilds the
// per-sweep coefficients from cst / gk. Partials state-major.
// part holds part_cap doubles (it also takes the slices of a split column
// pass, which the state pass then overwrites).
hipError_t launch_sweep_otf(hipStream_t s, const OtfModel& m, bool fp32, int K, int64_t N,
                            const double* cst, const double* gk, const double* h, double* logD,
                            double* part, size_t part_cap,
                            double* part_obj, unsigned* part_flags, int num_cus, int* grid_out);
// Rebuilds only the per-sweep coefficients (cf32 or cf64) from cst / gk.
hipError_t launch_otf_coefs(hipStream_t s, const OtfModel& m, bool fp32, int K, const double* cst,
                            const double* gk);
hipError_t launch_weights_otf(hipStream_t s, const OtfModel& m, int K, int64_t N, const double* f,
                              const double* logD, double* W);

// What the Hessian reads: kind 0 FP64 u; 1 FP32 u (widened); 2 packed
// mixed-precision matrix (cst = d_k, m0 = per-column shift); 3 model in FP32
// (otf.cf32 current); 4 model in FP64 (otf.cf64 current). Kinds 2 and 3 with
// K > 256 run on FP16 matrix cores (FP32 accumulation within a chunk).
struct HessSource {
  int kind = 0;  // as Mat::kind; 5: stored FP64 u on the FP16 matrix cores (K > 256);
                 // 6: stored FP64 u with FP32 exponentials (FP64 accumulation);
                 // 8: stored FP32 u on the FP16 matrix cores (K > 256)
  int num_cus = 256;  // sizes the sample chunks of the FP16-core path
  const void* u = nullptr;
  int64_t ld = 0;
  const double* m0 = nullptr;
  OtfModel otf;
  void* p16 = nullptr;  // kinds 3, 5, 8 with K > 256: the sample-tiled FP16 copy of P,
                        // K x p16_samples(K, N) halves
};
// samples of P held per super-chunk by the FP16-core Hessian: N rounded up to
// whole 32-sample tiles, capped at 4 GiB of FP16
int64_t p16_samples(int K, int64_t N);
hipError_t launch_hessian(hipStream_t s, const HessSource& hs, int K, int64_t N,
                          const double* cst, const double* gk, const double* logD,
                          const double* S, double* partials, int chunks, double* H);
// Two-pass FP64 sweep for any K (FP64 or FP32 u); grid returned in *grid_out.
int wide_grid(int64_t N, int num_cus);
hipError_t launch_sweep_wide(hipStream_t s, const void* u, bool f32, int64_t ld, int K, int64_t N,
                             const double* cst, const double* gk, const double* h, double* logD,
                             double* part, double* part_obj, unsigned* part_flags, int num_cus,
                             int* grid_out);
// Mixed precision (sweep32.hip).
bool sweep32_supported(int K);
hipError_t launch_pack_f32(hipStream_t s, const void* u, bool f32, int64_t ld, int K, int64_t N,
                           const double* c0, float* r, int64_t ldr, double* m0);
hipError_t launch_delta(hipStream_t s, int K, const double* f, const double* f0, double* d);
hipError_t launch_sweep32(hipStream_t s, const float* r, int64_t ld, int K, int64_t N,
                          const double* dk, const double* gk, const double* m0, double* logD,
                          double* part, double* part_obj, unsigned* part_flags, int num_cus,
                          int* grid_out);
// Newton direction on the reduced system (drop the first sampled state and
// the unsampled ones). A: workspace K*K doubles, idx: K ints. ok: device int.
hipError_t launch_newton_direction(hipStream_t s, int K, const int64_t* Nk, const double* H,
                                   const double* S, double* A, int* idx, double* d, int* ok);
// Largest reduced size the single-workgroup LDS solve takes.
int newton_lds_max_m();
// Blocked Cholesky solve of the same reduced system for any 0 < m < K; idx
// (m entries, the kept states) must be on the device; A holds
// newton_ws_doubles(K) doubles.
size_t newton_ws_doubles(int K);
// Blocked Cholesky A = L L^T of an SPD m x m matrix in place (A then holds L
// below the diagonal blocks' diagonals, Linv the inverses of the 64 x 64
// diagonal blocks) and y = L^{-1} b; *ok = 0 on a pivot that is not positive.
hipError_t launch_chol_factor_blocked(hipStream_t s, int m, double* A, double* b, double* y,
                                     double* Linv, int* ok);
// Asymptotic covariance of f (covariance.hip).
hipError_t launch_cov_consts(hipStream_t s, int K, const double* f, double* cst, double* gk,
                             double* S);
hipError_t launch_cov_gather(hipStream_t s, int K, int m, const int* idx, const int64_t* Nk,
                             const double* Mneg, double* A, double* b, double* Bm);
hipError_t launch_cov_solve(hipStream_t s, int m, int K, const double* A, const double* Linv,
                            double* Bm);
hipError_t launch_cov_theta(hipStream_t s, int m, int K, const double* Z, const double* Mneg,
                            double* Th, double* cov);
hipError_t launch_newton_direction_blocked(hipStream_t s, int K, int m, const int64_t* Nk,
                                           const double* H, const double* S, double* A,
                                           const int* idx, double* d, int* ok);
// u_kn = model_k(xi_n), K x N with row stride N, FP64 or (f32) rounded to
// FP32; d in {1, 2}.
hipError_t launch_model_energies(hipStream_t s, int K, int64_t N, int d, int model,
                                 const double* coef, const double* xi, void* u, bool f32);
// dst[i] = (double)src[i] for i < n (exact).
hipError_t launch_widen_f32(hipStream_t s, const float* src, int64_t n, double* dst);

}  // namespace bumbar

constexpr size_t kPinnedBytes = 16384;  // a context's pinned readback buffer

struct bumbar_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cus = 256;
  std::string err;
  void* pinned = nullptr;  // pinned host buffer of kPinnedBytes for small readbacks
  // optional timing of the unbinned sweep kernel (HIP events on ctx->stream)
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t events_used = 0;
  // private stream on which batches of binned steps are captured as graphs
  // (created on first use; nothing executes on it)
  hipStream_t cap_stream = nullptr;
  // this device's address of the library's fixed scratch array (bumbar_sweep_static)
  void* static_scratch = nullptr;
  // set while a solve runs as a fiber of a caller-driven server: instead of
  // blocking on a busy stream the solve hands control back to the server
  void (*yield)(void*) = nullptr;
  void* yield_arg = nullptr;
  // set by a server that fuses the small batches of its problems into one
  // launch: the batch is handed over instead of launched; the call returns
  // once the fused launch is queued and ctx->stream waits for it
  int (*post_small)(void* arg, const bumbar::SmallBatch& a) = nullptr;
  void* post_arg = nullptr;
  // cooperative batches allowed (cleared for server slots, whose streams run
  // concurrently, and after a cooperative launch failed)
  bool coop_ok = true;
};
