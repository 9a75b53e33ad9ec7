// bumbar_sweep_static: the single sweep of bumbar_sweep with its scratch
// buffers (per-state constants, per-workgroup partial sums, the finaliser's
// scalars) in a fixed device array of this file instead of a caller
// workspace, for callers that cannot allocate device memory.
//
// `scratch` below is a file-scope device array: its name is a host-side
// stand-in, not a device address. Its address on each device is taken once
// with hipGetSymbolAddress while that device is current (static_scratch_init,
// called from bumbar_create) and only that address is handed to kernels.
// Every call on a device shares the device's array; calls that overlap on one
// device race. Nothing in it has to start at zero: every sweep writes each
// partial before the finaliser reads it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "bumbar_impl.h"
#include "solver_internal.h"

namespace bumbar {

constexpr size_t kStaticScratchBytes = size_t(8) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Called with ctx->device current. Resolves the array's address on this
// device once per process and stores it in the context.
int static_scratch_init(bumbar_ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices) return BUMBAR_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) return BUMBAR_EDEVICE;
    g_scratch_ptr[ctx->device] = p;
  }
  ctx->static_scratch = g_scratch_ptr[ctx->device];
  return BUMBAR_OK;
}

// The subset of UnbinnedBufs a single sweep touches, carved from the array.
static bool carve_static(Arena& ar, UnbinnedBufs& B, int K, int64_t N, int num_cus) {
  B.K = K;
  B.N = N;
  B.cst = ar.take<double>(K);
  B.gk = ar.take<double>(K);
  B.lnNp = ar.take<double>(K);
  B.lnS = ar.take<double>(K);
  B.S = ar.take<double>(K);
  const int ch = robust_chunks(N);
  B.nparts_cap = std::max(sweep_max_grid(num_cus), ch);
  B.part = ar.take<double>((size_t)B.nparts_cap * K);
  B.partS = ar.take<double>((size_t)ch * K);
  B.part_obj = ar.take<double>(B.nparts_cap);
  B.part_flags = ar.take<unsigned>(B.nparts_cap);
  B.scal = ar.take<SweepScalars>(2);
  return !ar.overflow;
}

}  // namespace bumbar

using namespace bumbar;

extern "C" int bumbar_sweep_static(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K,
                                   int64_t N, int64_t ld, const int64_t* N_k, const double* f,
                                   double* f_new, double* log_D_n, double* S,
                                   double* sweep_stats) {
  if (!ctx) return BUMBAR_EINVAL;
  ctx->err.clear();
  if (!u_kn || !N_k || !f || !f_new || !log_D_n)
    return fail(ctx, BUMBAR_EINVAL, "NULL argument (u_kn, N_k, f, f_new and log_D_n are required)");
  if (K <= 0 || N <= 0) return fail(ctx, BUMBAR_EINVAL, "K and N must be positive");
  if (K > BUMBAR_STATIC_MAX_K || N > BUMBAR_STATIC_MAX_N)
    return fail(ctx, BUMBAR_EINVAL, "bumbar_sweep_static takes K <= %d and N <= %lld (got %d, %lld)",
                BUMBAR_STATIC_MAX_K, (long long)BUMBAR_STATIC_MAX_N, K, (long long)N);
  if (ld < N) return fail(ctx, BUMBAR_EINVAL, "row stride ld < N");
  if (u_dtype != BUMBAR_F64 && u_dtype != BUMBAR_F32)
    return fail(ctx, BUMBAR_EINVAL, "u_dtype must be BUMBAR_F64 or BUMBAR_F32");
  if (!ctx->static_scratch) return fail(ctx, BUMBAR_EDEVICE, "static scratch not resolved");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BUMBAR_EDEVICE, "hipSetDevice");
  Arena ar{reinterpret_cast<char*>(ctx->static_scratch), kStaticScratchBytes};
  UnbinnedBufs B;
  if (!carve_static(ar, B, K, N, ctx->num_cus))
    return fail(ctx, BUMBAR_ENOMEM, "static scratch of %zu bytes too small for K = %d, N = %lld",
                kStaticScratchBytes, K, (long long)N);
  Mat M;
  M.u = u_kn;
  M.kind = (u_dtype == BUMBAR_F32) ? 1 : 0;
  M.ld = ld;
  double* Sv = S ? S : B.S;
  // the same launches as bumbar_sweep: queued only, or with the scalars read
  // back and a flagged sweep redone on the robust path
  if (sweep_stats == nullptr && sweep_fast_supported(K))
    return sweep_queue(ctx, B, M, N, nullptr, N_k, f, f_new, log_D_n, B.lnS, Sv, B.scal);
  SweepScalars sc{};
  const int rc = sweep_at(ctx, B, M, N, nullptr, N_k, f, f_new, log_D_n, B.lnS, Sv, &sc, false,
                          nullptr);
  if (rc) return rc;
  if (sweep_stats) {
    sweep_stats[0] = sc.max_df;
    sweep_stats[1] = sc.rel_step;
    sweep_stats[2] = sc.objective;
    sweep_stats[3] = sc.grad_norm;
  }
  return BUMBAR_OK;
}
