/*
 * bumbar.h -- C ABI of the MI355X (gfx950) BU-MBAR solver library (libbumbar.so).
 *
 * Problem (Muller, Alesiani, Christiansen, "BU-MBAR: a hybrid solution
 * strategy for the MBAR equations", Section 2): K thermodynamic states, N
 * samples pooled from all states, N_k of them drawn in state k (sum N_k = N),
 * and the reduced energy u_kn of every sample n evaluated in every state k
 * (the paper's beta_k E_n, generalised to any reduced energy). The solver
 * returns the free energies f_k (gauge f_0 = 0) that solve the MBAR equations
 *     f_i = -log sum_n exp(-u_in) / sum_k N_k exp(f_k - u_kn),
 * the limit of infinitesimal bin width of the binned WHAM iteration, Eq. (1),
 * and optionally the weights W_nk = exp(f_k - u_kn) / sum_j N_j exp(f_j - u_jn).
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers on the context's device unless a
 *    parameter says "host". The caller allocates and owns all of them; the
 *    library never frees caller memory and never keeps a pointer past the
 *    call.
 *  - u_kn is K x N row-major (state-major: sample index n contiguous),
 *    element type given by a BUMBAR_F64 / BUMBAR_F32 code. Rows may be
 *    padded: ld >= N is the row stride in elements where a call takes one.
 *  - N_k is int64 on the device; states with N_k = 0 are allowed (they are
 *    excluded from the denominators and their f_k is filled from the
 *    MBAR formula).
 *  - u_kn = +inf is allowed (sample impossible in that state); NaN or -inf
 *    make the call fail with BUMBAR_EINVAL.
 *  - Work is issued on the context's HIP stream. Calls that return host
 *    scalars or statistics synchronise that stream before returning; the
 *    others return once their work is queued unless noted.
 *  - No call throws; each returns a status code and stores a message
 *    retrievable with bumbar_last_error().
 *  - A context is not thread-safe: use one context per host thread.
 */
#ifndef BUMBAR_H
#define BUMBAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define BUMBAR_OK 0
#define BUMBAR_EINVAL (-1)   /* bad shape, dtype, sum N_k != N, non-finite input, tol <= 0 */
#define BUMBAR_ENOMEM (-2)   /* workspace too small or host allocation failed             */
#define BUMBAR_EDEVICE (-3)  /* a HIP runtime call failed                                 */
#define BUMBAR_ENOTCONV (-4) /* iteration cap reached; the best f is still written        */
#define BUMBAR_ETOOBIG (-5)  /* request larger than the server's memory budget            */
#define BUMBAR_EBUSY (-6)    /* server has no free slot / ticket not finished              */

/* ---- codes ------------------------------------------------------------ */
#define BUMBAR_F64 0
#define BUMBAR_F32 1
/* The sample-major copy of u_kn (bumbar_sample_major), taken by bumbar_sweep
 * for 256 < K <= 1024: the same FP64 / FP32 elements transposed to N rows of
 * Kp = 64 J values (J the smallest of 5, 6, 8, 10, 12, 14, 16 with K <= 64 J;
 * states past K hold +inf), so that one sample
 * is one contiguous run of HBM. */
#define BUMBAR_F64_SMAJOR 2
#define BUMBAR_F32_SMAJOR 3

#define BUMBAR_PREC_FP64 0  /* every sweep in FP64                                       */
#define BUMBAR_PREC_MIXED 1 /* FP32 sweeps, FP64 accumulation/solve, FP64 refinement     */

#define BUMBAR_FINISH_NEWTON 0
#define BUMBAR_FINISH_SCI 1

#define BUMBAR_MODEL_NONE 0     /* bin representative = mean of the bin's u_kn           */
#define BUMBAR_MODEL_LINEAR 1   /* u_k(x) = c_k + sum_j a_kj x_j                         */
#define BUMBAR_MODEL_HARMONIC 2 /* u_k(x) = c_k + sum_j kappa_kj / 2 (x_j - x0_kj)^2     */

/* Bin representatives of Eq. (1) (bumbar_options.represent). CENTRE: the
 * model at the bin centre, evaluated inside the binned sweeps (needs a
 * model; the workspace holds only the P x d centres). MEAN: the mean of u_kn
 * over the bin's samples (needs an FP64 u_kn; the workspace holds K x P
 * representatives, P <= N). AUTO: CENTRE when a model is given, else MEAN;
 * the workspace is sized for both. */
#define BUMBAR_REPRESENT_AUTO 0
#define BUMBAR_REPRESENT_CENTRE 1
#define BUMBAR_REPRESENT_MEAN 2

/* Kernels of the FP64 unbinned sweeps (bumbar_plan.sweep). */
#define BUMBAR_SWEEP_REGISTER 0     /* K <= 256: register-tiled single pass (FP32 u
                                       widened on load)                                 */
#define BUMBAR_SWEEP_SAMPLE_MAJOR 1 /* 256 < K <= 1024: single pass over a sample-major
                                       copy of u in the workspace                       */
#define BUMBAR_SWEEP_TWO_PASS 2     /* two passes over the state-major u (K > 1024, or
                                       the copy switched off)                           */
#define BUMBAR_SWEEP_MODEL 3        /* energies from the model inside the kernels       */
/* The FP32 Newton stage of BUMBAR_PREC_MIXED (bumbar_plan.stage32). */
#define BUMBAR_STAGE32_NONE 0
#define BUMBAR_STAGE32_PACKED 1       /* r_kn = fp32(c0_k - u_kn - m0_n), K <= 256          */
#define BUMBAR_STAGE32_SAMPLE_MAJOR 2 /* FP32 arithmetic over the sample-major copy        */
#define BUMBAR_STAGE32_MODEL 3        /* the model evaluated in FP32                        */
#define BUMBAR_STAGE32_STORED 4       /* FP32 exponentials over FP32-stored u, K <= 256     */

typedef struct bumbar_ctx bumbar_ctx;

/* One phase-2 check of Algorithm 1 (Section 2). */
typedef struct {
  int64_t n;      /* nominal bin target n0 * inc^t before the decision   */
  int64_t P;      /* nonempty bins at n                                  */
  int64_t P_next; /* nonempty bins at n * inc                            */
  double s_n;     /* relative step, Eq. (2), at n                        */
  double s_next;  /* relative step, Eq. (2), at n * inc                  */
  int refine;     /* 1 if n was multiplied by inc (Eq. (3) test)         */
  int stop;       /* 1 if the binned stage ended after this check        */
} bumbar_check;

typedef struct {
  double tol;          /* finisher stops when a full Newton step has max_k |delta f_k| < tol
                          (kT; SCI finisher: the SCI step). Default 1e-10                */
  int precision;       /* BUMBAR_PREC_*                                                  */
  int binning;         /* 1: Algorithm 1 on the coordinates xi, then the finisher;
                          0: plain unbinned SCI then the finisher                        */
  int64_t n0;          /* initial nonempty-bin target (paper: 100)                       */
  double eps;          /* phase-1 stop on the relative step, Eq. (2) (paper: 1e-3)        */
  int64_t inc;         /* refinement factor (paper: 10)                                  */
  int n_intermediate;  /* SCI steps between refinement checks (paper: 20)                */
  int finisher;        /* BUMBAR_FINISH_NEWTON or BUMBAR_FINISH_SCI                       */
  int64_t max_iter;    /* cap on SCI steps of all stages (default 1e6)                   */
  int max_newton;      /* cap on finisher Newton steps (default 100)                     */
  double sci_switch;   /* plain mode: unbinned SCI until max |delta f| < sci_switch      */
  int replay_phase1;   /* schedule replay: phase-1 steps (used if replay_refine != NULL)  */
  const int* replay_refine; /* host; schedule replay: refine flag of each phase-2 check  */
  int n_replay;        /* number of entries in replay_refine                              */
  int profile;         /* 1: time every unbinned sweep kernel with HIP events (stats)      */
  double mixed_tol;    /* PREC_MIXED: Newton on the FP32 matrix until max |delta f| <
                          mixed_tol, then FP64 refinement to tol (default 1e-6)          */
  int represent;       /* bin representatives (BUMBAR_REPRESENT_*); default AUTO         */
  int graphs;          /* 1 (default): each batch of binned SCI steps queued between two
                          readbacks is captured once as a HIP graph (per batch shape and
                          level) and replayed for every later batch of that shape; 0: the
                          kernels are launched one by one. Same results to the bit.     */
  int sample_major;    /* 1 (default): for 256 < K <= 1024 a stored u_kn is copied once per
                          solve to a sample-major layout in the workspace (N Kp elements,
                          Kp as for BUMBAR_F64_SMAJOR, of the input type) and every unbinned sweep
                          reads the copy in one pass; 0: no copy, two-pass sweeps over
                          u_kn (FP64 only: PREC_MIXED with 256 < K needs the copy)         */
  int u_dtype;         /* element type of the u_kn bumbar_solve will get (BUMBAR_F64,
                          default, or BUMBAR_F32): the workspace queries size the copy
                          with it (an FP32 copy with a query for FP64 fits)              */
  int xi_dtype;        /* element type of the xi bumbar_solve will get (BUMBAR_F64,
                          default, or BUMBAR_F32): FP32 coordinates are widened (exactly)
                          into N d doubles of the workspace, which the queries then
                          include; a workspace sized for FP64 is too small for FP32 xi  */
  const char* trace_path; /* host string or NULL: append the solve's trace to this text
                          file (one line per phase-2 check of Algorithm 1: nominal n, bins
                          at n and n inc, the relative steps of Eq. (2), refine and stop;
                          then a summary line of stage lengths, finisher steps and stage
                          times); EINVAL if it cannot be written                      */
  int grid_batches;    /* 1: a batch of binned SCI steps on a level held in the
                          sample-major layout (256 < K <= 1024) runs as one cooperative
                          launch, with grid barriers between each step's sweep and its
                          per-state sums (the device must then run no other cooperative
                          kernel at the same time; server slots do not use it); 0
                          (default): per-step kernels, which are faster on MI355X    */
} bumbar_options;

typedef struct {
  int64_t phase1_iters;     /* binned SCI steps in phase 1                              */
  int64_t phase2_iters;     /* binned SCI steps after phase 1 (incl. probes)            */
  int64_t n_checks;         /* phase-2 checks performed                                 */
  int64_t finisher_steps;   /* finisher steps (Newton or SCI)                           */
  int64_t sci_fallbacks;    /* Newton steps replaced by an SCI step                      */
  int64_t unbinned_sweeps;  /* full K x N sweeps                                        */
  int64_t robust_sweeps;    /* sweeps redone on the two-pass underflow-safe path         */
  int64_t hessians;         /* K x K Hessian contractions                               */
  int64_t mixed_steps;      /* finisher steps taken on the FP32 packed matrix            */
  double final_step;        /* last applied max |delta f| (kT)                           */
  double grad_norm;         /* Euclidean norm of the MBAR gradient at the result         */
  double time_binning_ms;   /* histogram / width search                                 */
  double time_binned_ms;    /* binned SCI stages                                        */
  double time_final_ms;     /* unbinned finisher                                        */
  double sweep_kernel_ms;   /* profile = 1: summed duration of the unbinned sweep kernels */
  int64_t sweep_kernel_launches; /* profile = 1: number of timed sweep kernel launches   */
  bumbar_check* checks;     /* host, caller-owned, may be NULL: schedule of phase 2     */
  int checks_capacity;      /* entries available in checks                              */
  int64_t graph_batches;    /* batches of binned steps launched as HIP graphs            */
  int64_t grid_sweeps;      /* FP64 model sweeps done on the product-grid passes (2-D
                               harmonic windows whose factors form a grid)              */
  int64_t batched_steps;    /* binned SCI steps run inside single-workgroup batches (levels
                               of at most 512 bins, the matrix held in registers)       */
  int64_t damped_steps;     /* Newton steps accepted with alpha < 1 (the finisher stops
                               only after a full step, or a fresh full step below tol)  */
  int64_t coop_steps;       /* binned SCI steps run inside cooperative batches (levels
                               materialised sample-major, 256 < K <= 1024)              */
} bumbar_stats;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device` issuing work on `hip_stream`
 * (a hipStream_t; NULL = the default stream). */
int bumbar_create(bumbar_ctx** out, int device, void* hip_stream);
void bumbar_destroy(bumbar_ctx* ctx);
/* Message of the last failed call on ctx (never NULL; "" if none). */
const char* bumbar_last_error(const bumbar_ctx* ctx);
/* Library version string, "bumbar-gfx950 <version> src:<h>", where h is the
 * first 16 hex digits of the SHA-256 of the library's sources, this header
 * and the compiler flags it was built from. */
const char* bumbar_version(void);

/* Defaults: the paper's settings n0 = 100, eps = 1e-3, inc = 10,
 * n_intermediate = 20 (Section 2, after Algorithm 1), tol = 1e-10,
 * Newton finisher, FP64, binning off. */
void bumbar_default_options(bumbar_options* opt);

/* ---- workspace -------------------------------------------------------- */

/* Bytes of device workspace bumbar_solve needs for a K x N problem with
 * d-dimensional binning coordinates (d = 0 if no binning). With K > 256 and
 * the Newton finisher this includes the sample-tiled FP16 copy of P that the
 * FP16-core Hessian reads: 2 K min(N, 2^31 / K) bytes. */
int bumbar_query_workspace(const bumbar_ctx* ctx, int K, int64_t N, int d,
                           const bumbar_options* opt, size_t* bytes);

/* Bytes of device workspace bumbar_solve needs when u_kn is NULL (energies
 * from the model, d-dimensional coordinates, d in {1, 2}). opt NULL: enough
 * for a binned Newton solve at either precision, and for bumbar_sweep_model
 * and bumbar_hessian_model at either. With K > 256 and precision MIXED the
 * Newton Hessian holds a sample-tiled FP16 copy of P in the workspace:
 * 2 K min(N, 2^31 / K) bytes (longer problems are taken in super-chunks). */
int bumbar_query_workspace_model(const bumbar_ctx* ctx, int K, int64_t N, int d,
                                 const bumbar_options* opt, size_t* bytes);

/* ---- solve ------------------------------------------------------------ */

/*
 * Solve the MBAR equations (Eq. 1) by BU-MBAR (Algorithm 1): binned SCI
 * steps on successively finer bins of the coordinates xi, each level ended
 * by the relative-step tests of Eqs. (2) and (3), then the unbinned
 * finisher (Newton on the reduced system, Section 2).
 *  u_kn     K x N (row stride N), dtype u_dtype. With precision MIXED, an
 *           FP64 u_kn is packed to FP32 internally (in the workspace).
 *           NULL: the energies are the model's (HARMONIC or LINEAR, coef
 *           and xi required, d in {1, 2}), evaluated inside the kernels at
 *           every use and never stored; size the workspace with
 *           bumbar_query_workspace_model. With precision MIXED the Newton
 *           stage then runs on FP32 model sweeps (FP32 coordinates) before
 *           the FP64 refinement.
 *  N_k      K int64.
 *  xi       N x d binning coordinates (row-major), d in {1, 2}, element
 *           type xi_dtype (BUMBAR_F64 or BUMBAR_F32; FP32 is widened exactly
 *           to FP64 in the workspace, and the solve is then that of the
 *           widened coordinates); required when opt->binning = 1 or u_kn is
 *           NULL, else may be NULL.
 *  model    BUMBAR_MODEL_*; coef is K x (1 + 2d) float64 (layout in the
 *           model codes above), or NULL for BUMBAR_MODEL_NONE. With a model
 *           the bin representative is the model at the bin centre; without,
 *           the mean of u_kn over the bin's samples.
 *  f_init   K float64 starting point, or NULL for f = 0 (Algorithm 1 starts
 *           from 0; f_init is used only when binning = 0).
 *  f_k      K float64 output (gauge f_0 = 0).
 *  W_nk     N x K float64 output (sample-major) or NULL.
 *  log_D_n  N float64 output, ln sum_k N_k exp(f_k - u_kn), or NULL.
 *  stats    host, may be NULL.
 * Synchronises the stream. Returns BUMBAR_ENOTCONV (with f_k written) if
 * max_iter or max_newton is reached.
 */
int bumbar_solve(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N,
                 const int64_t* N_k, const void* xi, int xi_dtype, int d, int model,
                 const double* coef, const double* f_init, const bumbar_options* opt,
                 void* workspace, size_t ws_bytes, double* f_k, double* W_nk,
                 double* log_D_n, bumbar_stats* stats);

/*
 * What bumbar_solve would run for a problem of this shape and options,
 * decided on the host without touching a device (the solve and the
 * workspace queries take the same decisions): stored_u = 1 for a stored
 * u_kn of element type u_dtype, 0 for energies from the model; num_cus the
 * device's compute units (256 on MI355X; sizes the workspace). Returns
 * BUMBAR_EINVAL, with the reason in msg (host, may be NULL), for a
 * combination bumbar_solve refuses, e.g. PREC_MIXED with the SCI finisher,
 * with a stored u_kn and K > 1024, or with 256 < K <= 1024 and
 * sample_major = 0: mixed precision is never replaced by FP64 silently.
 */
typedef struct {
  int precision;          /* BUMBAR_PREC_MIXED if an FP32 Newton stage runs, else FP64      */
  int represent;          /* resolved bin representative (0 without binning)                */
  int sweep;              /* BUMBAR_SWEEP_*: the FP64 unbinned sweeps                        */
  int stage32;            /* BUMBAR_STAGE32_*: the FP32 stage                                */
  int fp32_binned;        /* 1: binned steps first run on the FP32 model sweep               */
  int hessian_fp16;       /* 1: the Newton Hessian runs on the FP16 matrix cores              */
  size_t copy_bytes;      /* sample-major copy of u_kn in the workspace (0: none)            */
  size_t workspace_bytes; /* workspace bumbar_solve needs                                     */
} bumbar_plan;
int bumbar_plan_solve(int num_cus, int stored_u, int u_dtype, int K, int64_t N, int d, int model,
                      const bumbar_options* opt, bumbar_plan* out, char* msg, size_t msg_len);

/* ---- uncertainty of f ------------------------------------------------- */

/*
 * Asymptotic covariance of the free energies at the solution f (gauge
 * f_0 = 0): cov[i * K + j] = Cov(f_i, f_j), K x K float64 row-major (device),
 * zero on row and column 0. The estimator is the large-sample covariance of
 * the MBAR estimate (Shirts and Chodera, J. Chem. Phys. 129, 124105 (2008)),
 *   Theta = W^T (I_N - W diag(N_k) W^T)^+ W,  W_nk = exp(f_k - u_kn - ln D_n),
 *   Cov(f_i, f_j) = (e_i - e_0)^T Theta (e_j - e_0);
 * the paper cites uncertainty estimates as related work (Section 1). It is
 * evaluated as K x K algebra: W^T W by the FP64 matrix cores (the Newton
 * Hessian's contraction), then a Cholesky solve with the reduced Hessian of
 * the sampled states. Unsampled states get their covariances too. u_kn is
 * state-major (row stride ld, FP64 or FP32), f the converged solution (e.g.
 * from bumbar_solve; ln D_n is recomputed from it). Workspace:
 * bumbar_query_workspace_covariance bytes. Synchronises. EINVAL if the
 * reduced Hessian is not positive definite (sampled states without overlap).
 */
int bumbar_query_workspace_covariance(const bumbar_ctx* ctx, int K, int64_t N, size_t* bytes);
int bumbar_covariance(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N,
                      int64_t ld, const int64_t* N_k, const double* f, void* workspace,
                      size_t ws_bytes, double* cov);

/* ---- single steps (the kernels of the solve, exposed for testing) ------ */

/*
 * One unbinned self-consistent iteration (Eq. (1) with one sample per bin):
 *   ln D_n   = ln sum_{k: N_k>0} N_k exp(f_k - u_kn)
 *   f_new_i  = -ln sum_n exp(-u_in - ln D_n),  then f_new -= f_new_0
 *   S_i      = sum_n N_i exp(f_i - u_in - ln D_n) (= N_i sum_n W_ni)
 * u_kn K x N with row stride ld >= N. f (K), outputs f_new (K), log_D_n (N,
 * may be NULL), S (K, may be NULL). sweep_stats (host, may be NULL) receives
 * {max_i |f_new_i - f_i|, relative step Eq. (2), sum_n ln D_n - sum_k N_k f_k,
 * Euclidean norm of S - N over sampled states}. The workspace must hold
 * bumbar_query_workspace(ctx, K, N, 0, NULL) bytes. Synchronises iff
 * sweep_stats != NULL.
 */
int bumbar_sweep(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N, int64_t ld,
                 const int64_t* N_k, const double* f, void* workspace, size_t ws_bytes,
                 double* f_new, double* log_D_n, double* S, double* sweep_stats);

/*
 * Hessian of the MBAR objective F(f) = sum_n ln D_n - sum_k N_k f_k at f:
 *   H_ij = delta_ij S_i - sum_n P_ni P_nj,  P_ni = N_i exp(f_i - u_in - ln D_n)
 * (the W W^T contraction; zero rows/columns for N_k = 0). log_D_n must be
 * ln D_n at f (e.g. from bumbar_sweep) and S the matching S. H is K x K
 * float64 row-major. Uses FP64 MFMA.
 */
int bumbar_hessian(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N,
                   int64_t ld, const int64_t* N_k, const double* f, const double* log_D_n,
                   const double* S, void* workspace, size_t ws_bytes, double* H);

/*
 * The same Hessian as the Newton steps build it for K > 256 (Section 2, the
 * derivative-based finisher; it only shapes the steps): P rounded to FP16
 * into a sample-tiled copy in the workspace, G = P P^T on the FP16 matrix
 * cores with FP32 sums inside a sample chunk and FP64 across chunks. Same
 * arguments as bumbar_hessian; K > 256 (else BUMBAR_EINVAL), u_dtype
 * BUMBAR_F64 or BUMBAR_F32. Workspace: bumbar_query_workspace(ctx, K, N, 0,
 * NULL) bytes. Does not synchronise.
 */
int bumbar_hessian_fp16(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N,
                        int64_t ld, const int64_t* N_k, const double* f, const double* log_D_n,
                        const double* S, void* workspace, size_t ws_bytes, double* H);

/*
 * The same single sweep and Hessian with u_kn taken from the model (the
 * on-the-fly kinds of bumbar_solve with u_kn = NULL): coef K x (1 + 2d),
 * xi N x d float64 (device). precision BUMBAR_PREC_FP64 evaluates the model
 * and the exponentials in FP64; BUMBAR_PREC_MIXED in FP32 (coordinates
 * rounded to FP32, log2-domain expanded quadratic, hardware exp2) with FP64
 * partial sums. Workspace: bumbar_query_workspace_model(ctx, K, N, d, NULL).
 * Both synchronise; an FP32 sweep whose sums leave the FP32 range returns
 * BUMBAR_EINVAL.
 */
int bumbar_sweep_model(bumbar_ctx* ctx, int K, int64_t N, int d, int model, const double* coef,
                       const double* xi, int precision, const int64_t* N_k, const double* f,
                       void* workspace, size_t ws_bytes, double* f_new, double* log_D_n,
                       double* S, double* sweep_stats);
int bumbar_hessian_model(bumbar_ctx* ctx, int K, int64_t N, int d, int model, const double* coef,
                         const double* xi, int precision, const int64_t* N_k, const double* f,
                         const double* log_D_n, const double* S, void* workspace,
                         size_t ws_bytes, double* H);

/*
 * The sample-major copy of a state-major K x N matrix (256 < K <= 1024,
 * u_dtype BUMBAR_F64 or BUMBAR_F32, row stride ld): element (k, n) is stored
 * at n Kp + k with Kp = 64 J, J the smallest of 5, 6, 8, 10, 12, 14, 16 with
 * K <= 64 J; entries k >= K are +inf (a state no
 * sample can visit). bumbar_sample_major_elems gives N Kp (or -1 where the
 * layout is not defined); bumbar_sample_major writes the copy to u_nk
 * (device, caller-allocated, that many elements of the input type).
 * Stream-ordered, does not synchronise. Pass the copy to bumbar_sweep with
 * u_dtype BUMBAR_F64_SMAJOR / BUMBAR_F32_SMAJOR. bumbar_solve makes such a
 * copy in its workspace by itself (bumbar_options.sample_major).
 */
int64_t bumbar_sample_major_elems(int K, int64_t N);
int bumbar_sample_major(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N,
                        int64_t ld, void* u_nk);

/* W_nk = exp(f_k - u_kn - ln D_n), N x K float64 (sample-major). */
int bumbar_weights(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N, int64_t ld,
                   const double* f, const double* log_D_n, double* W_nk);

/*
 * Binning for a target of n nonempty bins (Section 2, after Eq. (1)):
 * quantise xi (N x d float64) per dimension onto 32-bit integers anchored at
 * the minimum, find the width m (in quanta) by integer bisection for
 * max{m : g(m) >= n}, and build the histogram over the nonempty bins in
 * ascending cell order. Outputs (device, caller-sized for the worst case
 * N): cells (uint64, P entries), H (int64 counts, P entries), sample_bin
 * (int32, N entries, may be NULL); host outputs m_out, P_out. Synchronises.
 */
int bumbar_bin(bumbar_ctx* ctx, const double* xi, int64_t N, int d, int64_t n_target,
               void* workspace, size_t ws_bytes, uint64_t* m_out, int64_t* P_out,
               uint64_t* cells, int64_t* H, int32_t* sample_bin);

/*
 * Per-sample probabilities at a target state, Eqs. (5)-(6) (Section 3):
 *   p_n = exp(-u_target_n - ln D_n) / sum_m exp(-u_target_m - ln D_m).
 * u_target (N) and log_D_n (N) in, p (N) out. Synchronises.
 */
int bumbar_reweight(bumbar_ctx* ctx, const double* u_target, int64_t N, const double* log_D_n,
                    void* workspace, size_t ws_bytes, double* p);

/*
 * Free-energy surface on a regular grid of the coordinates (Section 3: the
 * surfaces of Fig. 1 from the probabilities of Eqs. (5)-(6)):
 *   F_b = -ln sum_{n in bin b} p_n,
 * bin b = b_0 nbins_1 + b_1 (d = 2; b = b_0 for d = 1) with
 *   b_j = floor((xi_nj - lo_j) * nbins_j / (hi_j - lo_j))   (FP64, this order).
 * Samples with some b_j outside [0, nbins_j) are left out; empty bins get
 * +inf. Each bin's p_n are added in increasing n within segments of at most
 * 1024 samples, then the segment sums in order, so F does not depend on the
 * launch. xi (N x d, FP64, d in {1, 2}) and p (N) in, F (nbins_0 * nbins_1)
 * out, all device; lo, hi, nbins: host arrays of d entries (finite lo < hi,
 * nbins >= 1, fewer than 2^32 bins; N < 2^32). The workspace must hold
 * bumbar_query_workspace_pmf bytes. Synchronises. EINVAL for a bad grid or
 * argument, ENOMEM for a short workspace.
 */
int bumbar_query_workspace_pmf(const bumbar_ctx* ctx, int64_t N, size_t* bytes);
int bumbar_pmf(bumbar_ctx* ctx, const double* xi, int64_t N, int d, const double* p,
               const double* lo, const double* hi, const int* nbins, void* workspace,
               size_t ws_bytes, double* F);

/* ---- allocation-free sweep -------------------------------------------- */

/*
 * bumbar_sweep without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, kernels and results as bumbar_sweep,
 * except that log_D_n is required (it also carries ln D between the passes
 * of the FP32-input path). Its scratch (per-state constants, per-workgroup
 * partial sums, the finaliser's scalars) is a fixed 8 MiB device array of
 * the library, one per device, resolved when a context is created: the call
 * performs no device allocation of any kind. Limits: K <= BUMBAR_STATIC_MAX_K
 * and N <= BUMBAR_STATIC_MAX_N, else BUMBAR_EINVAL. Every call on a device
 * shares that device's array and leaves its last contents there, so calls
 * that overlap on one device (two streams, two host threads) race: serialise
 * them. Synchronises iff sweep_stats != NULL, as bumbar_sweep.
 */
#define BUMBAR_STATIC_MAX_K 256
#define BUMBAR_STATIC_MAX_N ((int64_t)1 << 22)
int bumbar_sweep_static(bumbar_ctx* ctx, const void* u_kn, int u_dtype, int K, int64_t N,
                        int64_t ld, const int64_t* N_k, const double* f, double* f_new,
                        double* log_D_n, double* S, double* sweep_stats);

/* ---- batched serving ---------------------------------------------------
 *
 * A server keeps up to max_active MBAR problems resident on one device and
 * solves them concurrently (one HIP stream and context per active slot, so
 * the kernels of different problems overlap on the GPU); new requests are
 * admitted in arrival order as soon as a slot is free and the problem's
 * device footprint (its u_kn, inputs and solver workspace) fits in the
 * server's memory arena, which is reserved once at creation. Each problem is
 * solved by exactly the kernels and launch shapes of bumbar_solve, so its
 * result is bitwise the same alone and in the mix.
 *
 * Two ways of driving the slots: worker threads (caller_driven = 0, one host
 * thread per slot), or none at all (caller_driven = 1): then every admitted
 * solve is a fiber (a user-level context on its own stack) that advances
 * only inside bumbar_server_progress (and bumbar_server_wait, which calls
 * it), on the calling thread. A fiber runs until its stream is busy with
 * the kernels it queued, then hands control to the next one, so the
 * problems' kernels still overlap on the device.
 *
 * A caller-driven server may also fuse (fuse = 1): the batches of binned
 * self-consistent steps (Eq. (1) with the bin counts, Algorithm 1) that
 * its problems reach on levels small enough for one workgroup are not
 * launched per problem; each tick gathers them into a device work list and
 * replays one captured HIP graph (the list's upload, then one kernel whose
 * fixed grid walks the list), so a single launch advances every resident
 * problem that is in such a batch. Each item runs the same code as its own
 * launch would: results stay bitwise the same alone and in the mix.
 */
typedef struct bumbar_server bumbar_server;

typedef struct {
  int device;               /* HIP device                                              */
  size_t hbm_budget_bytes;  /* device memory reserved for resident requests            */
  int max_active;           /* problems solved concurrently (>= 1)                     */
  int caller_driven;        /* 1: no worker threads; the caller's progress() calls
                               advance the problems (all server calls but submit, poll,
                               result and counters from the creating thread)          */
  int fuse;                 /* 1: fused launches of the small binned batches (needs
                               caller_driven = 1; EINVAL otherwise); 0: off           */
} bumbar_server_options;

typedef struct {
  int K;
  int64_t N;
  const void* u_kn;     /* host K x N of type u_dtype, or NULL: energies from the model   */
  int u_dtype;          /* BUMBAR_F64 or BUMBAR_F32: host u_kn, or the materialised u     */
  const int64_t* N_k;   /* host, K entries                                               */
  const void* xi;       /* host N x d coordinates (binning and/or model), or NULL        */
  int xi_dtype;         /* BUMBAR_F64 or BUMBAR_F32                                      */
  int d;                /* coordinate dimension (0 if xi is NULL)                         */
  int model;            /* BUMBAR_MODEL_*                                                */
  const double* coef;   /* host K x (1 + 2d) model coefficients, or NULL                  */
  int materialize;      /* with u_kn = NULL: 1 evaluates the model once into a resident
                           device u_kn of type u_dtype (counted in the footprint) and
                           solves that stored matrix; 0 evaluates it inside the kernels */
  bumbar_options opt;   /* solve options                                                 */
} bumbar_request;

#define BUMBAR_TICKET_QUEUED 0
#define BUMBAR_TICKET_RUNNING 1
#define BUMBAR_TICKET_DONE 2
#define BUMBAR_TICKET_FAILED 3

/* Reserve the memory arena and set up max_active slots (with a worker
 * thread each unless caller_driven). */
int bumbar_server_create(const bumbar_server_options* opt, bumbar_server** out);
/* Queue a request. The host arrays it points to must stay valid until the
 * ticket is DONE or FAILED. BUMBAR_ETOOBIG if its footprint exceeds the
 * whole arena. */
int bumbar_server_submit(bumbar_server* srv, const bumbar_request* req, uint64_t* ticket);
/* State of a ticket (BUMBAR_TICKET_*); EINVAL for an unknown ticket. */
int bumbar_server_poll(bumbar_server* srv, uint64_t ticket, int* state);
/* Block until the ticket is DONE or FAILED (caller-driven: calls
 * bumbar_server_progress until it is). */
int bumbar_server_wait(bumbar_server* srv, uint64_t ticket);
/* One tick of a caller-driven server: admit queued requests into free slots
 * in arrival order while their footprints fit, resume every admitted solve
 * until it waits on its stream or finishes, and retire the finished ones
 * (f read back, arena block released). *n_done (may be NULL) receives the
 * number of tickets that finished in this tick. Does not block on the
 * device. EINVAL for a threaded server or a call from another thread than
 * the creating one. */
int bumbar_server_progress(bumbar_server* srv, int* n_done);
/* Result of a finished ticket: f_k (host, K entries, or NULL), statistics
 * (host, may be NULL; its checks array is not filled), latency from
 * submission to completion in ms, and the solve's status code. The ticket
 * is released: a second call (or a poll) returns EINVAL. EBUSY if the ticket
 * has not finished (it is then kept). */
int bumbar_server_result(bumbar_server* srv, uint64_t ticket, double* f_k_host,
                         bumbar_stats* stats, double* latency_ms, int* status);
/* Counters (each pointer may be NULL): completed requests, largest number
 * of problems on the device at once, largest arena use in bytes, and the
 * requests that had to wait at the head of the queue, with a slot free,
 * until enough of the arena was released (admission bound by memory). */
int bumbar_server_counters(bumbar_server* srv, int64_t* completed, int64_t* peak_active,
                           size_t* peak_bytes, int64_t* mem_waits);
/* Fused launches of a fusing server so far, and the batches they ran
 * (items / launches is the mean number of problems advanced per launch);
 * both 0 for a server without fuse. */
int bumbar_server_fused_counters(bumbar_server* srv, int64_t* launches, int64_t* items);
/* Let running requests finish, fail the ones still queued (status
 * BUMBAR_EBUSY), stop the slots and release the arena. */
void bumbar_server_destroy(bumbar_server* srv);

/* u_kn = model_k(xi_n) on the device (K x N, row stride N): the reduced
 * energies of the LINEAR / HARMONIC models (layout of coef as in
 * bumbar_solve) for N coordinates xi (N x d float64, d in {1, 2}),
 * evaluated in FP64 and stored as u_dtype (BUMBAR_F64, or BUMBAR_F32:
 * rounded once); every pointer is device memory owned by the caller. Any
 * potential common to all states is left out, since it cancels in Eq. (1).
 * Stream-ordered on the context's stream (does not synchronise); EINVAL for
 * a bad argument. */
int bumbar_model_energies(bumbar_ctx* ctx, int K, int64_t N, int d, int model,
                          const double* coef, const double* xi, int u_dtype, void* u_kn);

#ifdef __cplusplus
}
#endif

#endif /* BUMBAR_H */
