// Host-side planning of bumbar_solve: which kernels run (FP64 sweep form,
// FP32 stage, Hessian source) and which workspace buffers are carved for
// them, from the call's shapes and options alone. The solve, the workspace
// queries and bumbar_plan_solve all go through make_plan / carve_plan, so a
// path never launches with a buffer its plan did not carve, and an option
// combination the kernels do not cover is refused with BUMBAR_EINVAL instead
// of being run some other way.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>

#include "bumbar_impl.h"
#include "solver_internal.h"

namespace bumbar {

size_t Plan::copy_bytes() const {
  return copy ? smaj_elems(K, N) * (copy_f32 ? sizeof(float) : sizeof(double)) : 0;
}

int make_plan(const bumbar_options& opt, bool otf, int u_dtype, int K, int64_t N, int d,
              int model, Plan* p, std::string* msg) {
  auto bad = [msg](const char* m) {
    *msg = m;
    return BUMBAR_EINVAL;
  };
  *p = Plan();
  if (K <= 0 || N <= 0) return bad("K and N must be positive");
  if (!otf && u_dtype != BUMBAR_F64 && u_dtype != BUMBAR_F32)
    return bad("u_dtype must be BUMBAR_F64 or BUMBAR_F32");
  // model = -1: not known yet (the workspace queries), sized for either representative
  const bool model_known = model != -1;
  if (model_known && model != BUMBAR_MODEL_NONE && model != BUMBAR_MODEL_LINEAR &&
      model != BUMBAR_MODEL_HARMONIC)
    return bad("unknown model code");
  if (otf && (model == BUMBAR_MODEL_NONE || d < 1 || d > 2))
    return bad("u_kn = NULL needs a model, its coefficients and xi (d in {1, 2})");
  if (!(opt.tol > 0.0)) return bad("tol must be > 0");
  if (opt.precision != BUMBAR_PREC_FP64 && opt.precision != BUMBAR_PREC_MIXED)
    return bad("unknown precision");
  if (opt.finisher != BUMBAR_FINISH_NEWTON && opt.finisher != BUMBAR_FINISH_SCI)
    return bad("unknown finisher");
  if (opt.binning && (d < 1 || d > 2))
    return bad("binning needs coordinates xi with d in {1, 2}");
  if (opt.binning && (opt.n0 < 2 || opt.inc < 2 || opt.n_intermediate < 0 || !(opt.eps > 0.0)))
    return bad("invalid binning settings");
  if (opt.represent < BUMBAR_REPRESENT_AUTO || opt.represent > BUMBAR_REPRESENT_MEAN)
    return bad("unknown bin representative");
  if (opt.xi_dtype != BUMBAR_F64 && opt.xi_dtype != BUMBAR_F32)
    return bad("xi_dtype must be BUMBAR_F64 or BUMBAR_F32");
  p->otf = otf;
  p->u_dtype = otf ? BUMBAR_F64 : u_dtype;
  p->K = K;
  p->N = N;
  p->d = d;
  p->binning = opt.binning != 0;
  p->xi_wide = d > 0 && opt.xi_dtype == BUMBAR_F32;
  p->rep = opt.represent != BUMBAR_REPRESENT_AUTO || !model_known
               ? opt.represent
               : (model != BUMBAR_MODEL_NONE ? BUMBAR_REPRESENT_CENTRE : BUMBAR_REPRESENT_MEAN);
  if (p->binning && p->rep == BUMBAR_REPRESENT_CENTRE && model == BUMBAR_MODEL_NONE)
    return bad("bin-centre representatives need a model");
  if (p->binning && p->rep == BUMBAR_REPRESENT_MEAN && (otf || u_dtype != BUMBAR_F64))
    return bad("mean bin representatives need FP64 u_kn (or give a model)");
  p->mixed = opt.precision == BUMBAR_PREC_MIXED;
  if (p->mixed && opt.finisher != BUMBAR_FINISH_NEWTON)
    return bad("mixed precision needs the Newton finisher (its FP32 stage is a Newton stage)");
  const bool f32 = p->u_dtype == BUMBAR_F32;
  // the FP64 sweeps
  if (otf)
    p->sweep = BUMBAR_SWEEP_MODEL;
  else if (sweep_fast_supported(K))
    p->sweep = BUMBAR_SWEEP_REGISTER;
  else if (sweep_smaj_supported(K) && opt.sample_major)
    p->sweep = BUMBAR_SWEEP_SAMPLE_MAJOR;
  else
    p->sweep = BUMBAR_SWEEP_TWO_PASS;
  // the FP32 stage
  if (p->mixed) {
    if (otf)
      p->stage32 = BUMBAR_STAGE32_MODEL;
    else if (sweep_fast_supported(K))
      // FP32 storage is read as it is (FP32 exponentials, no copy); FP64
      // storage is packed once to FP32 differences
      p->stage32 = f32 ? BUMBAR_STAGE32_STORED : BUMBAR_STAGE32_PACKED;
    else if (p->sweep == BUMBAR_SWEEP_SAMPLE_MAJOR)
      p->stage32 = BUMBAR_STAGE32_SAMPLE_MAJOR;
    else if (sweep_smaj_supported(K))
      return bad("mixed precision with 256 < K <= 1024 runs on the sample-major copy "
                 "(options.sample_major = 0 switches the copy off)");
    else
      return bad("mixed precision with a stored u_kn takes K <= 1024");
  }
  p->copy = p->sweep == BUMBAR_SWEEP_SAMPLE_MAJOR;
  p->copy_f32 = f32;
  // binned stage buffers: stored representatives (K x P) where the
  // register-tiled sweep takes K (its binned steps are one launch each) or
  // for MEAN; bin centres for the model sweeps otherwise
  if (p->binning) {
    if (otf || p->rep == BUMBAR_REPRESENT_CENTRE) {
      // bin centres: the model at the centres, materialised for levels of up
      // to otf_ubar_cap bins (K <= 256), else evaluated inside the sweeps
      p->bb_ubar = false;
      p->bb_cen = true;
      p->bb_otf_cap = otf_ubar_cap(K, N);
    } else {
      // bin means of the stored u: every level materialised (an unresolved
      // AUTO also carves the centres)
      p->bb_ubar = true;
      p->bb_cen = p->rep != BUMBAR_REPRESENT_MEAN;
      p->bb_otf_cap = 0;
    }
    // on the fly with K > 256 a binned step is a model sweep over K x P: the
    // FP32 stage first runs it in FP32 on FP32 centres. Not for stored u:
    // there the binned stage only provides the Newton start, and on ladders
    // with energies of ~1e3 kT the FP32 relative steps never pass eps (the
    // c2 ladder spent 4000 FP32 steps, ~0.4 s, before the FP64 rerun).
    p->bb_cen_f32 = otf && p->mixed && K > 256 && p->bb_cen;
    p->fp32_binned = p->bb_cen_f32;
  }
  p->x_packed = p->stage32 == BUMBAR_STAGE32_PACKED;
  p->o_bufs = otf || (p->binning && p->bb_cen);
  // Newton Hessian sources of stored u (it only shapes the steps; the FP64
  // sweeps decide the fixed point): the FP16 matrix cores for K > 256, FP32
  // exponentials with FP64 accumulation for FP64 u with K <= 256
  if (!otf) {
    p->hess_kind = K > 256 ? (f32 ? 8 : 5) : (f32 ? 1 : 6);
    p->hess_kind32 = p->stage32 == BUMBAR_STAGE32_PACKED ? 2 : p->hess_kind;
  }
  // the FP16-core Newton Hessian (stored u with K > 256, the FP32 model with
  // K > 256) reads P from a sample-tiled FP16 copy filled once per Hessian
  // (at most 4 GiB; longer problems are taken in super-chunks)
  if (opt.finisher == BUMBAR_FINISH_NEWTON && K > 256)
    p->p16 = otf ? p->mixed : true;
  return BUMBAR_OK;
}

void carve_plan(Arena& ar, const Plan& p, int num_cus, PlanBufs* pb) {
  pb->B.carve(ar, p.K, p.N, num_cus);
  if (p.binning)
    pb->BB.carve(ar, p.K, p.N, p.d, num_cus, p.bb_ubar, p.bb_cen, p.bb_cen_f32, p.bb_otf_cap);
  if (p.x_packed) pb->X.carve(ar, p.K, p.N);
  if (p.o_bufs) pb->O.carve(ar, p.K, p.N, p.d);
  if (p.copy) pb->copy = ar.take<char>(p.copy_bytes());
  if (p.xi_wide) pb->xi64 = ar.take<double>((size_t)p.N * p.d);
  if (p.p16) pb->p16 = ar.take<char>((size_t)p.K * (size_t)p16_samples(p.K, p.N) * 2);
}

}  // namespace bumbar

using namespace bumbar;

extern "C" int bumbar_plan_solve(int num_cus, int stored_u, int u_dtype, int K, int64_t N, int d,
                                 int model, const bumbar_options* opt_in, bumbar_plan* out,
                                 char* msg, size_t msg_len) {
  if (msg && msg_len) msg[0] = '\0';
  if (!out || num_cus < 1) return BUMBAR_EINVAL;
  bumbar_options opt;
  if (opt_in)
    opt = *opt_in;
  else
    bumbar_default_options(&opt);
  Plan p;
  std::string why;
  const int rc = make_plan(opt, stored_u == 0, u_dtype, K, N, d, model, &p, &why);
  if (rc) {
    if (msg && msg_len) snprintf(msg, msg_len, "%s", why.c_str());
    return rc;
  }
  Arena ar;
  PlanBufs pb;
  carve_plan(ar, p, num_cus, &pb);
  std::memset(out, 0, sizeof(*out));
  out->precision = p.mixed ? BUMBAR_PREC_MIXED : BUMBAR_PREC_FP64;
  out->represent = p.binning ? p.rep : 0;
  out->sweep = p.sweep;
  out->stage32 = p.stage32;
  out->fp32_binned = p.fp32_binned ? 1 : 0;
  const int hk = p.mixed ? p.hess_kind32 : p.hess_kind;
  out->hessian_fp16 = (hk == 5 || hk == 8 || (p.otf && p.mixed && K > 256)) ? 1 : 0;
  out->copy_bytes = p.copy_bytes();
  out->workspace_bytes = ar.off + 256;
  return BUMBAR_OK;
}
