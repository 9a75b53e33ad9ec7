/*
 * bumbar_oracle.c -- plain FP64 CPU oracle for BU-MBAR.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, obviously-correct reference
 * against which the GPU solver is checked. Only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load it. It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Everything is double precision, written as plain loops in the order the
 * paper states the equations. Sums over samples use Neumaier compensation so
 * that the oracle's own rounding is far below the 1e-9 kT parity tolerance.
 * OpenMP (if enabled) only splits independent outer loops (one sample or one
 * state per iteration); every individual sum runs in a fixed order on one
 * thread, so results do not depend on the thread count.
 *
 * Source of each function (Muller, Alesiani, Christiansen, "BU-MBAR: a hybrid
 * solution strategy for the MBAR equations"):
 *   - Section 2, Eq. (1): the binned WHAM self-consistent iteration (SCI).
 *     Its limit of one sample per bin is the unbinned MBAR/UWHAM iteration,
 *     with the bin energy term beta_i E_p replaced by a general reduced energy
 *     u_in and the histogram count by 1.
 *   - Section 2, text after Eq. (1): binning with a uniform width chosen as the
 *     largest width that still gives at least n nonempty bins; empty bins are
 *     skipped.
 *   - Section 2, Eq. (2): relative step width s.
 *   - Section 2, Eq. (3) and Algorithm 1: the adaptive refinement schedule.
 *   - Section 2 (derivative-based strategies) and Section 3 (final unbinned
 *     quasi-Newton iterations): the Newton finisher on the convex MBAR
 *     objective, whose gradient is the MBAR equation.
 *   - Section 3, Eqs. (5)-(6): per-sample reweighting probabilities.
 *
 * Readings where the paper is silent or inconsistent are listed in the
 * comment of each function that depends on them.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOTCONV (-4)

/* ------------------------------------------------------------------------ */
/* Compensated summation (Neumaier's improvement of Kahan summation).        */
/* ------------------------------------------------------------------------ */
typedef struct {
  double s;
  double c;
} nsum;

static void ns_init(nsum* a) { a->s = 0.0; a->c = 0.0; }

static void ns_add(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}

static double ns_val(const nsum* a) { return a->s + a->c; }

/* log(sum_j exp(x_j)) over x[j*stride], j < n, with the exact maximum as the
 * shift. Entries equal to -inf contribute nothing; an all -inf input gives
 * -inf. */
static double lse_strided(int64_t n, const double* x, int64_t stride) {
  double m = -INFINITY;
  for (int64_t j = 0; j < n; ++j) {
    double v = x[j * stride];
    if (v > m) m = v;
  }
  if (m == -INFINITY) return -INFINITY;
  nsum s;
  ns_init(&s);
  for (int64_t j = 0; j < n; ++j) ns_add(&s, exp(x[j * stride] - m));
  return m + log(ns_val(&s));
}

/* ------------------------------------------------------------------------ */
/* One self-consistent iteration of Eq. (1), binned or unbinned.             */
/* ------------------------------------------------------------------------ */

/*
 * ln D_p = log sum_{k: N_k > 0} N_k exp(f_k - ubar_kp)          (denominator
 * of Eq. (1), with beta_k E_p generalised to the reduced energy ubar_kp).
 *
 * ubar is K x P row-major (state-major); for unbinned data P = N and
 * ubar = u. States with N_k = 0 do not contribute to the denominator.
 */
int orc_log_denominator(int K, int64_t P, const double* ubar, const int64_t* Nk,
                        const double* f, double* logD) {
  if (K <= 0 || P < 0) return ORC_EINVAL;
  double* lnN = (double*)malloc(sizeof(double) * (size_t)K);
  if (!lnN) return ORC_ENOMEM;
  for (int k = 0; k < K; ++k) lnN[k] = Nk[k] > 0 ? log((double)Nk[k]) : -INFINITY;
#pragma omp parallel
  {
    double* a = (double*)malloc(sizeof(double) * (size_t)K);
#pragma omp for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
      for (int k = 0; k < K; ++k)
        a[k] = Nk[k] > 0 ? lnN[k] + f[k] - ubar[(int64_t)k * P + p] : -INFINITY;
      logD[p] = lse_strided(K, a, 1);
    }
    free(a);
  }
  free(lnN);
  return ORC_OK;
}

/*
 * One SCI step, Eq. (1):
 *   f_new_i = - log sum_p H_p exp(-ubar_ip) / D_p
 *           = - LSE_p( ln H_p - ubar_ip - ln D_p ).
 * logH == NULL means every H_p = 1 (unbinned MBAR, one sample per "bin").
 * Reading: f has no normalisation in Eq. (1); the gauge f_0 = 0 is applied
 * after every step so that the relative step of Eq. (2) is well defined.
 * logD_out (length P) may be NULL; if given it receives ln D_p evaluated at
 * the input f.
 */
int orc_sci_step(int K, int64_t P, const double* ubar, const double* logH,
                 const int64_t* Nk, const double* f, double* f_new, double* logD_out) {
  if (K <= 0 || P <= 0) return ORC_EINVAL;
  double* logD = logD_out ? logD_out : (double*)malloc(sizeof(double) * (size_t)P);
  if (!logD) return ORC_ENOMEM;
  int rc = orc_log_denominator(K, P, ubar, Nk, f, logD);
  if (rc) {
    if (!logD_out) free(logD);
    return rc;
  }
#pragma omp parallel
  {
    double* t = (double*)malloc(sizeof(double) * (size_t)P);
#pragma omp for schedule(static)
    for (int i = 0; i < K; ++i) {
      for (int64_t p = 0; p < P; ++p)
        t[p] = (logH ? logH[p] : 0.0) - ubar[(int64_t)i * P + p] - logD[p];
      f_new[i] = -lse_strided(P, t, 1);
    }
    free(t);
  }
  double g0 = f_new[0];
  for (int i = 0; i < K; ++i) f_new[i] -= g0;
  if (!logD_out) free(logD);
  return ORC_OK;
}

/*
 * Relative step width, Eq. (2): s = max_i |f_new_i / f_old_i - 1|.
 * Reading: the gauge state 0 is excluded (its value is 0 by construction);
 * where f_old_i = 0 the term is 0 if f_new_i = 0 and +inf otherwise, so the
 * first step from f = 0 never satisfies the phase-1 test.
 */
double orc_rel_step(int K, const double* f_new, const double* f_old) {
  double s = 0.0;
  for (int i = 1; i < K; ++i) {
    double r;
    if (f_old[i] != 0.0)
      r = fabs(f_new[i] / f_old[i] - 1.0);
    else
      r = (f_new[i] == 0.0) ? 0.0 : INFINITY;
    if (r > s || r != r) s = r;
  }
  return s;
}

/* ------------------------------------------------------------------------ */
/* Unbinned MBAR quantities (UWHAM limit of Eq. (1)).                        */
/* ------------------------------------------------------------------------ */

/* W_nk = exp(f_k - u_kn - ln D_n), written N x K (sample-major). */
int orc_weights(int K, int64_t N, const double* u, const int64_t* Nk, const double* f,
                double* W) {
  double* logD = (double*)malloc(sizeof(double) * (size_t)N);
  if (!logD) return ORC_ENOMEM;
  int rc = orc_log_denominator(K, N, u, Nk, f, logD);
  if (rc) { free(logD); return rc; }
#pragma omp parallel for schedule(static)
  for (int64_t n = 0; n < N; ++n)
    for (int k = 0; k < K; ++k) W[n * K + k] = exp(f[k] - u[(int64_t)k * N + n] - logD[n]);
  free(logD);
  return ORC_OK;
}

/*
 * Objective whose stationary point is the MBAR solution:
 *   F(f) = sum_n ln D_n - sum_k N_k f_k.
 * Gradient g_i = N_i (sum_n W_ni - 1) for N_i > 0 and 0 otherwise.
 * Either output pointer may be NULL.
 */
int orc_objective_gradient(int K, int64_t N, const double* u, const int64_t* Nk,
                           const double* f, double* F_out, double* g) {
  double* logD = (double*)malloc(sizeof(double) * (size_t)N);
  if (!logD) return ORC_ENOMEM;
  int rc = orc_log_denominator(K, N, u, Nk, f, logD);
  if (rc) { free(logD); return rc; }
  if (F_out) {
    nsum a;
    ns_init(&a);
    for (int64_t n = 0; n < N; ++n) ns_add(&a, logD[n]);
    for (int k = 0; k < K; ++k) ns_add(&a, -(double)Nk[k] * f[k]);
    *F_out = ns_val(&a);
  }
  if (g) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < K; ++i) {
      if (Nk[i] <= 0) { g[i] = 0.0; continue; }
      nsum s;
      ns_init(&s);
      for (int64_t n = 0; n < N; ++n) ns_add(&s, exp(f[i] - u[(int64_t)i * N + n] - logD[n]));
      g[i] = (double)Nk[i] * (ns_val(&s) - 1.0);
    }
  }
  free(logD);
  return ORC_OK;
}

/*
 * Hessian of F:
 *   H_ij = N_i delta_ij sum_n W_ni - N_i N_j sum_n W_ni W_nj
 * (rows and columns of N_k = 0 states are zero). Dense K x K, row-major.
 */
int orc_hessian(int K, int64_t N, const double* u, const int64_t* Nk, const double* f,
                double* H) {
  double* W = (double*)malloc(sizeof(double) * (size_t)N * (size_t)K);
  if (!W) return ORC_ENOMEM;
  int rc = orc_weights(K, N, u, Nk, f, W);
  if (rc) { free(W); return rc; }
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < K; ++i) {
    for (int j = 0; j < K; ++j) {
      if (Nk[i] <= 0 || Nk[j] <= 0) { H[i * K + j] = 0.0; continue; }
      nsum s;
      ns_init(&s);
      for (int64_t n = 0; n < N; ++n) ns_add(&s, W[n * K + i] * W[n * K + j]);
      double v = -(double)Nk[i] * (double)Nk[j] * ns_val(&s);
      if (i == j) {
        nsum d;
        ns_init(&d);
        for (int64_t n = 0; n < N; ++n) ns_add(&d, W[n * K + i]);
        v += (double)Nk[i] * ns_val(&d);
      }
      H[i * K + j] = v;
    }
  }
  free(W);
  return ORC_OK;
}

/* Dense Cholesky A = L L^T in place (lower triangle), n x n row-major.
 * Returns 0 on success, -1 if A is not numerically positive definite. */
static int cholesky(int n, double* A) {
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0)) return -1;
    double l = sqrt(d);
    A[j * n + j] = l;
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = v / l;
    }
  }
  return 0;
}

static void cholesky_solve(int n, const double* L, double* b) {
  for (int i = 0; i < n; ++i) {
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= L[i * n + k] * b[k];
    b[i] = v / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double v = b[i];
    for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * b[k];
    b[i] = v / L[i * n + i];
  }
}

/*
 * Newton direction on the reduced system. The Hessian annihilates the
 * constant vector over sampled states (gauge freedom), so the first sampled
 * state and every N_k = 0 state are removed: solve H_RR d_R = -g_R, d = 0
 * elsewhere. Returns 0, or -1 if the reduced Hessian is not positive definite
 * (disconnected overlap or a degenerate problem).
 */
int orc_newton_direction(int K, const int64_t* Nk, const double* H, const double* g,
                         double* d) {
  int* idx = (int*)malloc(sizeof(int) * (size_t)K);
  int r = -1, m = 0;
  for (int k = 0; k < K; ++k) {
    d[k] = 0.0;
    if (Nk[k] <= 0) continue;
    if (r < 0) { r = k; continue; }
    idx[m++] = k;
  }
  if (m == 0) { free(idx); return 0; }
  double* A = (double*)malloc(sizeof(double) * (size_t)m * (size_t)m);
  double* b = (double*)malloc(sizeof(double) * (size_t)m);
  for (int a = 0; a < m; ++a) {
    b[a] = -g[idx[a]];
    for (int c = 0; c < m; ++c) A[a * m + c] = H[idx[a] * K + idx[c]];
  }
  int ok = cholesky(m, A);
  if (ok == 0) {
    cholesky_solve(m, A, b);
    for (int a = 0; a < m; ++a) d[idx[a]] = b[a];
  }
  free(A);
  free(b);
  free(idx);
  return ok;
}

/* Fill f_k of the unsampled states (N_k = 0) from the SCI formula at the
 * current f, then apply the gauge f_0 = 0. Sampled states are unchanged
 * except for the common shift. */
static int fill_unsampled_and_gauge(int K, int64_t N, const double* u, const int64_t* Nk,
                                    double* f) {
  int any = 0;
  for (int k = 0; k < K; ++k)
    if (Nk[k] <= 0) any = 1;
  if (any) {
    double* fs = (double*)malloc(sizeof(double) * (size_t)K);
    double* logD = (double*)malloc(sizeof(double) * (size_t)N);
    double* t = (double*)malloc(sizeof(double) * (size_t)N);
    orc_log_denominator(K, N, u, Nk, f, logD);
    for (int k = 0; k < K; ++k) {
      if (Nk[k] > 0) { fs[k] = f[k]; continue; }
      for (int64_t n = 0; n < N; ++n) t[n] = -u[(int64_t)k * N + n] - logD[n];
      fs[k] = -lse_strided(N, t, 1);
    }
    memcpy(f, fs, sizeof(double) * (size_t)K);
    free(fs);
    free(logD);
    free(t);
  }
  double g0 = f[0];
  for (int k = 0; k < K; ++k) f[k] -= g0;
  return ORC_OK;
}

static double norm2(int K, const double* g) {
  nsum s;
  ns_init(&s);
  for (int k = 0; k < K; ++k) ns_add(&s, g[k] * g[k]);
  return sqrt(ns_val(&s));
}

/*
 * Derivative-based finisher on unbinned data (Section 2: derivative-based
 * strategies converge quadratically near the solution; Section 3: the last
 * iterations run a quasi-Newton scheme on unbinned data).
 * Reading (the paper names no specific scheme or tolerance): full Newton on
 * the reduced system; a trial step f + alpha d (alpha = 1, 1/2, ... , 2^-10)
 * is accepted when it lowers the Euclidean norm of the gradient; if no trial
 * step is accepted, or the reduced Hessian is not positive definite, one
 * unbinned SCI step is taken instead. Stops on a full Newton step: an
 * accepted alpha = 1 step with max_k |delta f_k| < tol, or a full step
 * max_k |d_k| < tol that is not accepted (the gradient norm has reached its
 * rounding floor). A damped or SCI step never ends the loop: its size does
 * not bound the distance to the solution. Returns the number of steps in
 * *steps_out.
 */
int orc_newton_finish(int K, int64_t N, const double* u, const int64_t* Nk, double* f,
                      double tol, int max_steps, int* steps_out, int* sci_fallbacks_out) {
  double* g = (double*)malloc(sizeof(double) * (size_t)K);
  double* g2 = (double*)malloc(sizeof(double) * (size_t)K);
  double* H = (double*)malloc(sizeof(double) * (size_t)K * (size_t)K);
  double* d = (double*)malloc(sizeof(double) * (size_t)K);
  double* ft = (double*)malloc(sizeof(double) * (size_t)K);
  int steps = 0, fallbacks = 0, rc = ORC_ENOTCONV;
  fill_unsampled_and_gauge(K, N, u, Nk, f);
  for (; steps < max_steps;) {
    orc_objective_gradient(K, N, u, Nk, f, NULL, g);
    double gn = norm2(K, g);
    orc_hessian(K, N, u, Nk, f, H);
    int accepted = 0, full = 0, have_dir = 0;
    double maxstep = 0.0, full_step = INFINITY;
    if (orc_newton_direction(K, Nk, H, g, d) == 0) {
      have_dir = 1;
      full_step = 0.0;
      for (int k = 0; k < K; ++k)
        if (fabs(d[k]) > full_step || d[k] != d[k]) full_step = fabs(d[k]);
      double alpha = 1.0;
      for (int t = 0; t <= 10; ++t, alpha *= 0.5) {
        for (int k = 0; k < K; ++k) ft[k] = f[k] + alpha * d[k];
        fill_unsampled_and_gauge(K, N, u, Nk, ft);
        orc_objective_gradient(K, N, u, Nk, ft, NULL, g2);
        if (norm2(K, g2) < gn) { accepted = 1; full = t == 0; break; }
      }
    }
    if (!accepted && have_dir && full_step < tol) { rc = ORC_OK; break; }
    if (!accepted) {
      orc_sci_step(K, N, u, NULL, Nk, f, ft, NULL);
      fill_unsampled_and_gauge(K, N, u, Nk, ft);
      ++fallbacks;
    }
    for (int k = 0; k < K; ++k) {
      double s = fabs(ft[k] - f[k]);
      if (s > maxstep || s != s) maxstep = s;
      f[k] = ft[k];
    }
    ++steps;
    if (full && maxstep < tol) { rc = ORC_OK; break; }
  }
  if (steps_out) *steps_out = steps;
  if (sci_fallbacks_out) *sci_fallbacks_out = fallbacks;
  free(g); free(g2); free(H); free(d); free(ft);
  return rc;
}

/*
 * Certified unbinned MBAR solution (the quantity the binned-to-unbinned
 * method converges to; Section 2: the unbinned equations are the limit of
 * infinitesimal bin width). Plain SCI from f_init until the step is below
 * sci_switch (or sci_max steps), then the Newton finisher to newton_tol.
 * residual_out receives max_k |SCI(f)_k - f_k| at the result.
 */
int orc_solve_mbar(int K, int64_t N, const double* u, const int64_t* Nk,
                   const double* f_init, double sci_switch, int sci_max, double newton_tol,
                   int newton_max, double* f, int* sci_steps_out, int* newton_steps_out,
                   double* residual_out) {
  if (K <= 0 || N <= 0) return ORC_EINVAL;
  int64_t tot = 0;
  for (int k = 0; k < K; ++k) {
    if (Nk[k] < 0) return ORC_EINVAL;
    tot += Nk[k];
  }
  if (tot != N) return ORC_EINVAL;
  double* fn = (double*)malloc(sizeof(double) * (size_t)K);
  for (int k = 0; k < K; ++k) f[k] = f_init ? f_init[k] - f_init[0] : 0.0;
  int sci = 0;
  for (; sci < sci_max; ++sci) {
    orc_sci_step(K, N, u, NULL, Nk, f, fn, NULL);
    double mx = 0.0;
    for (int k = 0; k < K; ++k) {
      double s = fabs(fn[k] - f[k]);
      if (s > mx || s != s) mx = s;
      f[k] = fn[k];
    }
    if (mx < sci_switch) { ++sci; break; }
  }
  int nsteps = 0, fb = 0;
  int rc = orc_newton_finish(K, N, u, Nk, f, newton_tol, newton_max, &nsteps, &fb);
  orc_sci_step(K, N, u, NULL, Nk, f, fn, NULL);
  double res = 0.0;
  for (int k = 0; k < K; ++k) {
    double s = fabs(fn[k] - f[k]);
    if (s > res || s != s) res = s;
  }
  if (sci_steps_out) *sci_steps_out = sci;
  if (newton_steps_out) *newton_steps_out = nsteps;
  if (residual_out) *residual_out = res;
  free(fn);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Binning (Section 2, text after Eq. (1)).                                  */
/* ------------------------------------------------------------------------ */

/*
 * Quantise each coordinate dimension onto 32-bit integers anchored at the
 * data minimum:
 *   lo = min xi, hi = max xi, scale = (2^32 - 1) / (hi - lo)  (0 if hi = lo),
 *   q  = min(floor((xi - lo) * scale), 2^32 - 1).
 * The subtraction and the multiplication are separate IEEE operations (this
 * file is compiled without floating-point contraction). xi is N x d
 * row-major; q is N x d. lo and scale (length d) are outputs.
 * Reading: the paper does not fix the bin origin or how the width is
 * represented; a uniform width of m quanta anchored at the minimum makes the
 * nonempty-bin count an exact integer function of m.
 */
int orc_quantize(int64_t N, int d, const double* xi, uint32_t* q, double* lo, double* scale) {
  if (N <= 0 || d < 1 || d > 2) return ORC_EINVAL;
  for (int j = 0; j < d; ++j) {
    double a = xi[j], b = xi[j];
    for (int64_t n = 0; n < N; ++n) {
      double v = xi[n * d + j];
      if (!(v == v) || isinf(v)) return ORC_EINVAL;
      if (v < a) a = v;
      if (v > b) b = v;
    }
    lo[j] = a;
    scale[j] = (b > a) ? 4294967295.0 / (b - a) : 0.0;
    for (int64_t n = 0; n < N; ++n) {
      double diff = xi[n * d + j] - a;
      double prod = diff * scale[j];
      double fl = floor(prod);
      if (fl > 4294967295.0) fl = 4294967295.0;
      q[n * d + j] = (uint32_t)fl;
    }
  }
  return ORC_OK;
}

/* Cell id of a quantised point for a width of m quanta. 1-D: q / m.
 * 2-D: row-major with the first coordinate fastest,
 *   (q_0 / m) + (q_1 / m) * (floor((2^32 - 1) / m) + 1). */
static uint64_t cell_of(int d, const uint32_t* qn, uint64_t m) {
  if (d == 1) return (uint64_t)qn[0] / m;
  uint64_t stride = 4294967295ull / m + 1ull;
  return (uint64_t)qn[0] / m + ((uint64_t)qn[1] / m) * stride;
}

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

/* g(m): the number of nonempty bins (distinct cells) for a width of m quanta.
 * Computed by sorting all cell ids and counting distinct values. */
int64_t orc_nonempty_bins(int64_t N, int d, const uint32_t* q, uint64_t m) {
  if (m == 0) return -1;
  uint64_t* c = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
  if (!c) return -1;
  for (int64_t n = 0; n < N; ++n) c[n] = cell_of(d, q + n * d, m);
  qsort(c, (size_t)N, sizeof(uint64_t), cmp_u64);
  int64_t g = N > 0 ? 1 : 0;
  for (int64_t n = 1; n < N; ++n) g += (c[n] != c[n - 1]);
  free(c);
  return g;
}

/*
 * Width for a target of n nonempty bins: w*(n) = max { w : n <= g(w) }.
 * Reading: g is not monotone in w, so the maximum is defined by this integer
 * bisection on m in [1, 2^32] with the invariant g(lo) >= n > g(hi)
 * (g(2^32) = 1): mid = lo + (hi - lo) / 2, keep the half that preserves the
 * invariant, stop at hi = lo + 1 and return lo. If even m = 1 gives fewer
 * than n bins (fewer distinct quantised values than n), m = 1 is returned:
 * every distinct value then sits in its own bin. Requires n >= 2.
 */
int orc_width_search(int64_t N, int d, const uint32_t* q, int64_t n_target, uint64_t* m_out,
                     int64_t* g_out, int* probes_out) {
  if (n_target < 2 || N <= 0) return ORC_EINVAL;
  int probes = 1;
  int64_t g1 = orc_nonempty_bins(N, d, q, 1);
  if (g1 < n_target) {
    *m_out = 1;
    if (g_out) *g_out = g1;
    if (probes_out) *probes_out = probes;
    return ORC_OK;
  }
  uint64_t lo = 1, hi = 4294967296ull;
  int64_t glo = g1;
  while (hi - lo > 1) {
    uint64_t mid = lo + (hi - lo) / 2;
    int64_t gm = orc_nonempty_bins(N, d, q, mid);
    ++probes;
    if (gm >= n_target) {
      lo = mid;
      glo = gm;
    } else {
      hi = mid;
    }
  }
  *m_out = lo;
  if (g_out) *g_out = glo;
  if (probes_out) *probes_out = probes;
  return ORC_OK;
}

/*
 * Histogram over the nonempty bins for width m: bins are the distinct cell ids
 * in ascending order; H[p] counts the samples in bin p; sample_bin[n] is the
 * bin index of sample n (may be NULL). cells_out (length >= n_act) may be
 * NULL. Returns the number of nonempty bins, or -1.
 */
int64_t orc_histogram(int64_t N, int d, const uint32_t* q, uint64_t m, uint64_t* cells_out,
                      int64_t* H, int32_t* sample_bin) {
  uint64_t* c = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
  uint64_t* s = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
  if (!c || !s) { free(c); free(s); return -1; }
  for (int64_t n = 0; n < N; ++n) c[n] = s[n] = cell_of(d, q + n * d, m);
  qsort(s, (size_t)N, sizeof(uint64_t), cmp_u64);
  int64_t P = 0;
  for (int64_t n = 0; n < N; ++n) {
    if (n == 0 || s[n] != s[n - 1]) {
      s[P] = s[n];
      H[P] = 0;
      ++P;
    }
    H[P - 1] += 1;
  }
  if (cells_out) memcpy(cells_out, s, sizeof(uint64_t) * (size_t)P);
  if (sample_bin) {
    for (int64_t n = 0; n < N; ++n) {
      int64_t a = 0, b = P - 1;
      while (a < b) {
        int64_t mid = a + (b - a) / 2;
        if (s[mid] < c[n]) a = mid + 1; else b = mid;
      }
      sample_bin[n] = (int32_t)a;
    }
  }
  free(c);
  free(s);
  return P;
}

/* Reduced-energy models for bin representatives. */
#define ORC_MODEL_LINEAR 1   /* u_k(x) = c_k + sum_j a_kj x_j                       */
#define ORC_MODEL_HARMONIC 2 /* u_k(x) = c_k + sum_j kappa_kj / 2 (x_j - x0_kj)^2    */

/* Coefficients per state: coef[k*(1+2d) + 0] = c_k; LINEAR: a_kj at 1 + j;
 * HARMONIC: kappa_kj at 1 + 2j and x0_kj at 2 + 2j. */
static double model_eval(int type, int d, const double* ck, const double* x) {
  double v = ck[0];
  for (int j = 0; j < d; ++j) {
    if (type == ORC_MODEL_LINEAR) {
      v += ck[1 + j] * x[j];
    } else {
      double dx = x[j] - ck[2 + 2 * j];
      v += 0.5 * ck[1 + 2 * j] * dx * dx;
    }
  }
  return v;
}

/*
 * Bin representatives, K x P row-major.
 * CENTRE (model given): ubar_kp = u_k(centre of bin p), the bin centre E_p of
 *   Eq. (1) generalised: centre_j = lo_j + (cell_j + 1/2) * m / scale_j
 *   (lo_j when scale_j = 0).
 * MEAN (model == NULL): ubar_kp = (1/H_p) sum_{n in p} u_kn.
 * Reading: for a general u_kn matrix there is no bin centre energy, so the
 * mean over the bin's members is used; with one sample per bin both give the
 * sample's own u_kn.
 */
int orc_represent(int K, int64_t N, int d, const double* u, int model_type, const double* coef,
                  const double* lo, const double* scale, uint64_t m, int64_t P,
                  const uint64_t* cells, const int64_t* H, const int32_t* sample_bin,
                  double* ubar) {
  if (model_type == ORC_MODEL_LINEAR || model_type == ORC_MODEL_HARMONIC) {
    uint64_t stride = 4294967295ull / m + 1ull;
    for (int64_t p = 0; p < P; ++p) {
      uint64_t cc[2];
      if (d == 1) {
        cc[0] = cells[p];
      } else {
        cc[0] = cells[p] % stride;
        cc[1] = cells[p] / stride;
      }
      double x[2];
      for (int j = 0; j < d; ++j)
        x[j] = scale[j] > 0.0 ? lo[j] + ((double)cc[j] + 0.5) * (double)m / scale[j] : lo[j];
      for (int k = 0; k < K; ++k)
        ubar[(int64_t)k * P + p] = model_eval(model_type, d, coef + (int64_t)k * (1 + 2 * d), x);
    }
    return ORC_OK;
  }
  if (!u || !sample_bin) return ORC_EINVAL;
  nsum* acc = (nsum*)malloc(sizeof(nsum) * (size_t)P);
  for (int k = 0; k < K; ++k) {
    for (int64_t p = 0; p < P; ++p) ns_init(&acc[p]);
    for (int64_t n = 0; n < N; ++n) ns_add(&acc[sample_bin[n]], u[(int64_t)k * N + n]);
    for (int64_t p = 0; p < P; ++p) ubar[(int64_t)k * P + p] = ns_val(&acc[p]) / (double)H[p];
  }
  free(acc);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (BU-MBAR) followed by the unbinned finisher.                  */
/* ------------------------------------------------------------------------ */

typedef struct {
  int64_t n;     /* nominal target */
  uint64_t m;    /* width in quanta */
  int64_t P;     /* nonempty bins */
  double* ubar;  /* K x P */
  double* logH;  /* P */
} level_t;

static void level_free(level_t* L) {
  free(L->ubar);
  free(L->logH);
  L->ubar = NULL;
  L->logH = NULL;
}

static int level_build(level_t* L, int64_t n_target, int K, int64_t N, int d, const double* u,
                       const uint32_t* q, int model_type, const double* coef, const double* lo,
                       const double* scale) {
  uint64_t m;
  int64_t g;
  int rc = orc_width_search(N, d, q, n_target, &m, &g, NULL);
  if (rc) return rc;
  uint64_t* cells = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
  int64_t* H = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
  int32_t* sb = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  int64_t P = orc_histogram(N, d, q, m, cells, H, sb);
  L->n = n_target;
  L->m = m;
  L->P = P;
  L->ubar = (double*)malloc(sizeof(double) * (size_t)K * (size_t)P);
  L->logH = (double*)malloc(sizeof(double) * (size_t)P);
  for (int64_t p = 0; p < P; ++p) L->logH[p] = log((double)H[p]);
  rc = orc_represent(K, N, d, u, model_type, coef, lo, scale, m, P, cells, H, sb, L->ubar);
  free(cells);
  free(H);
  free(sb);
  return rc;
}

/* One record per phase-2 check of Algorithm 1. */
typedef struct {
  int64_t n;        /* nominal bin target before the decision      */
  int64_t P;        /* nonempty bins at n                          */
  int64_t P_next;   /* nonempty bins at n * inc                    */
  double s_n;       /* Eq. (2) at n                                */
  double s_next;    /* Eq. (2) at n * inc                          */
  int refine;       /* 1 if n was multiplied by inc                */
  int stop;         /* 1 if the loop ended after this check        */
} orc_check_t;

/*
 * Algorithm 1 with the following readings of the pseudo-code:
 *  - SCI(f, n) is ONE application of Eq. (1) with the binning for target n
 *    (the pseudo-code computes the relative step between successive calls).
 *  - In phase 2 the probes f_new and f_next are not discarded: f <- f_next
 *    when the bins are refined, otherwise f <- f_new.
 *  - n is the nominal target n0 * inc^t in the Eq. (3) test and in the
 *    termination test 2 * inc * n > N; the comparisons are strict as printed.
 *  - Guard against a loop that cannot progress: if the width for n * inc is
 *    the same as for n (identical binning), the bins are refined at once.
 *  - Every binned SCI counts toward max_iter; reaching it returns ENOTCONV.
 * After the loop ends, the finisher runs on unbinned data until the applied
 * update is below tol (finisher: 0 = Newton as in orc_newton_finish,
 * 1 = plain unbinned SCI).
 * If replay_refine is non-NULL, phase 1 runs exactly replay_phase1 steps and
 * check c refines iff replay_refine[c] != 0 (schedule replay for parity of
 * another implementation's trajectory); the computed s values are still
 * reported.
 * checks (capacity max_checks) receives the phase-2 schedule; counts[0..3] =
 * {phase-1 SCIs, phase-2 SCIs (all binned steps after phase 1), number of
 * checks, finisher steps}. f_binned (may be NULL) receives f at the end of
 * the binned stage.
 */
int orc_bumbar(int K, int64_t N, const double* u, const int64_t* Nk, int d, const double* xi,
               int model_type, const double* coef, int64_t n0, double eps, int64_t inc,
               int n_int, double tol, int finisher, int64_t max_iter, int replay_phase1,
               const int* replay_refine, int n_replay, double* f, double* f_binned,
               orc_check_t* checks, int max_checks, int64_t* counts) {
  if (K <= 0 || N <= 0 || d < 1 || d > 2 || n0 < 2 || inc < 2 || n_int < 0) return ORC_EINVAL;
  int64_t tot = 0;
  for (int k = 0; k < K; ++k) tot += Nk[k];
  if (tot != N) return ORC_EINVAL;
  uint32_t* q = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)N * (size_t)d);
  double lo[2], scale[2];
  int rc = orc_quantize(N, d, xi, q, lo, scale);
  if (rc) { free(q); return rc; }
  double* fn = (double*)malloc(sizeof(double) * (size_t)K);
  double* fx = (double*)malloc(sizeof(double) * (size_t)K);
  for (int k = 0; k < K; ++k) f[k] = 0.0;
  int64_t it1 = 0, it2 = 0;
  int nchk = 0;
  rc = ORC_OK;

  /* Phase 1: iterate at n0 until the relative step is below eps. */
  int64_t n = n0;
  level_t cur = {0}, nxt = {0};
  level_build(&cur, n, K, N, d, u, q, model_type, coef, lo, scale);
  for (;;) {
    if (it1 + it2 >= max_iter) { rc = ORC_ENOTCONV; break; }
    orc_sci_step(K, cur.P, cur.ubar, cur.logH, Nk, f, fn, NULL);
    double s = orc_rel_step(K, fn, f);
    memcpy(f, fn, sizeof(double) * (size_t)K);
    ++it1;
    if (replay_refine ? (it1 >= replay_phase1) : (s < eps)) break;
  }

  /* Phase 2. */
  if (rc == ORC_OK) {
    n = n * inc;
    level_free(&cur);
    level_build(&cur, n, K, N, d, u, q, model_type, coef, lo, scale);
    level_build(&nxt, n * inc, K, N, d, u, q, model_type, coef, lo, scale);
    for (;;) {
      if (it1 + it2 + n_int + 2 > max_iter) { rc = ORC_ENOTCONV; break; }
      for (int i = 0; i < n_int; ++i) {
        orc_sci_step(K, cur.P, cur.ubar, cur.logH, Nk, f, fn, NULL);
        memcpy(f, fn, sizeof(double) * (size_t)K);
      }
      orc_sci_step(K, cur.P, cur.ubar, cur.logH, Nk, f, fn, NULL);
      double s_n = orc_rel_step(K, fn, f);
      orc_sci_step(K, nxt.P, nxt.ubar, nxt.logH, Nk, f, fx, NULL);
      double s_next = orc_rel_step(K, fx, f);
      it2 += n_int + 2;
      int refine;
      if (replay_refine)
        refine = (nchk < n_replay) ? replay_refine[nchk] != 0 : 0;
      else
        refine = (2.0 * s_next > (double)inc * s_n) || (nxt.m == cur.m);
      int stop = 0;
      orc_check_t rec;
      rec.n = n;
      rec.P = cur.P;
      rec.P_next = nxt.P;
      rec.s_n = s_n;
      rec.s_next = s_next;
      rec.refine = refine;
      if (refine) {
        memcpy(f, fx, sizeof(double) * (size_t)K);
        n = n * inc;
        if (2 * inc * n > N) stop = 1;
      } else {
        memcpy(f, fn, sizeof(double) * (size_t)K);
      }
      rec.stop = stop;
      if (nchk < max_checks) checks[nchk] = rec;
      ++nchk;
      if (stop) break;
      if (replay_refine && nchk >= n_replay) break;
      if (refine) {
        level_free(&cur);
        cur = nxt;
        nxt.ubar = NULL;
        nxt.logH = NULL;
        level_build(&nxt, n * inc, K, N, d, u, q, model_type, coef, lo, scale);
      }
    }
  }
  level_free(&cur);
  level_free(&nxt);
  if (f_binned) memcpy(f_binned, f, sizeof(double) * (size_t)K);

  /* Final stage on unbinned data. */
  int64_t fin = 0;
  if (rc == ORC_OK) {
    if (finisher == 0) {
      int st = 0, fb = 0;
      rc = orc_newton_finish(K, N, u, Nk, f, tol, 200, &st, &fb);
      fin = st;
    } else {
      for (;;) {
        if (it1 + it2 + fin >= max_iter) { rc = ORC_ENOTCONV; break; }
        orc_sci_step(K, N, u, NULL, Nk, f, fn, NULL);
        double mx = 0.0;
        for (int k = 0; k < K; ++k) {
          double s = fabs(fn[k] - f[k]);
          if (s > mx || s != s) mx = s;
        }
        memcpy(f, fn, sizeof(double) * (size_t)K);
        ++fin;
        if (mx < tol) break;
      }
    }
  }
  if (counts) {
    counts[0] = it1;
    counts[1] = it2;
    counts[2] = nchk;
    counts[3] = fin;
  }
  free(q);
  free(fn);
  free(fx);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Reweighting, Section 3, Eqs. (5)-(6).                                     */
/* ------------------------------------------------------------------------ */

/*
 * p_n proportional to exp(-u_target_n) / sum_m N_m exp(f_m - u_mn), normalised
 * to sum to one. Reading: Eq. (6) as printed is circular (C is the sum of the
 * p_i that already contain 1/C); C is taken as the sum of the unnormalised
 * terms, which is the only value that makes the p_n a probability
 * distribution. logD is ln D_n at the solution (orc_log_denominator).
 */
int orc_reweight(int64_t N, const double* u_target, const double* logD, double* p) {
  if (N <= 0) return ORC_EINVAL;
  double m = -INFINITY;
  for (int64_t n = 0; n < N; ++n) {
    double v = -u_target[n] - logD[n];
    if (v > m) m = v;
  }
  nsum s;
  ns_init(&s);
  for (int64_t n = 0; n < N; ++n) {
    p[n] = exp(-u_target[n] - logD[n] - m);
    ns_add(&s, p[n]);
  }
  double C = ns_val(&s);
  for (int64_t n = 0; n < N; ++n) p[n] /= C;
  return ORC_OK;
}

/* Free-energy surface on a regular grid (Section 3: the surfaces of Fig. 1,
 * from the probabilities of Eqs. (5)-(6)): F_b = -ln sum_{n in bin b} p_n with
 * bin b = b_0 nb_1 + b_1 (b = b_0 for d = 1) and
 * b_j = floor((xi_nj - lo_j) * nb_j / (hi_j - lo_j)); samples outside the grid
 * are left out, bins without probability get +inf. The p_n of a bin are added
 * in increasing n. */
int orc_pmf(int64_t N, int d, const double* xi, const double* p, const double* lo,
            const double* hi, const int* nb, double* F) {
  if (N <= 0 || (d != 1 && d != 2)) return ORC_EINVAL;
  int64_t total = 1;
  for (int j = 0; j < d; ++j) {
    if (nb[j] < 1 || !(hi[j] > lo[j])) return ORC_EINVAL;
    total *= nb[j];
  }
  double* acc = (double*)calloc((size_t)total, sizeof(double));
  char* hit = (char*)calloc((size_t)total, 1);
  if (!acc || !hit) {
    free(acc);
    free(hit);
    return ORC_EINVAL;
  }
  for (int64_t n = 0; n < N; ++n) {
    int64_t b = 0;
    int in = 1;
    for (int j = 0; j < d; ++j) {
      const double bj = floor((xi[n * d + j] - lo[j]) * (double)nb[j] / (hi[j] - lo[j]));
      if (!(bj >= 0.0 && bj < (double)nb[j])) {
        in = 0;
        break;
      }
      b = b * nb[j] + (int64_t)bj;
    }
    if (!in) continue;
    acc[b] += p[n];
    hit[b] = 1;
  }
  for (int64_t b = 0; b < total; ++b) F[b] = hit[b] ? -log(acc[b]) : INFINITY;
  free(acc);
  free(hit);
  return ORC_OK;
}

/* Size of the check record, so that a binding can verify its layout. */
int orc_check_record_size(void) { return (int)sizeof(orc_check_t); }
