"""Plain FP64 CPU oracle for BU-MBAR -- TEST INFRASTRUCTURE ONLY.

This package wraps ``bumbar_oracle.c`` (plain C, double precision) with
ctypes and numpy. Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the GPU library never does, and this
package never imports the GPU library. The two share no code: the only
module both sides use is ``synth`` (seeded input generators, none of the
method's arithmetic).

Every function cites the passage of the paper (Muller, Alesiani,
Christiansen, "BU-MBAR: a hybrid solution strategy for the MBAR equations")
that it follows; see ``bumbar_oracle.c`` for the readings of ambiguous
passages.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bumbar_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODEL_NONE = 0
MODEL_LINEAR = 1
MODEL_HARMONIC = 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no floating-point contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-std=c99", "-D_DEFAULT_SOURCE", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class CheckRecord(C.Structure):
    _fields_ = [("n", C.c_int64), ("P", C.c_int64), ("P_next", C.c_int64),
                ("s_n", C.c_double), ("s_next", C.c_double), ("refine", C.c_int),
                ("stop", C.c_int)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = C.CDLL(_LIB)
    dp, ip64, up32, up64, i32p = (C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                  C.POINTER(C.c_int32))
    lib.orc_log_denominator.argtypes = [C.c_int, C.c_int64, dp, ip64, dp, dp]
    lib.orc_sci_step.argtypes = [C.c_int, C.c_int64, dp, dp, ip64, dp, dp, dp]
    lib.orc_rel_step.argtypes = [C.c_int, dp, dp]
    lib.orc_rel_step.restype = C.c_double
    lib.orc_weights.argtypes = [C.c_int, C.c_int64, dp, ip64, dp, dp]
    lib.orc_objective_gradient.argtypes = [C.c_int, C.c_int64, dp, ip64, dp, dp, dp]
    lib.orc_hessian.argtypes = [C.c_int, C.c_int64, dp, ip64, dp, dp]
    lib.orc_newton_direction.argtypes = [C.c_int, ip64, dp, dp, dp]
    lib.orc_newton_finish.argtypes = [C.c_int, C.c_int64, dp, ip64, dp, C.c_double, C.c_int,
                                      C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.orc_solve_mbar.argtypes = [C.c_int, C.c_int64, dp, ip64, dp, C.c_double, C.c_int,
                                   C.c_double, C.c_int, dp, C.POINTER(C.c_int),
                                   C.POINTER(C.c_int), dp]
    lib.orc_quantize.argtypes = [C.c_int64, C.c_int, dp, up32, dp, dp]
    lib.orc_nonempty_bins.argtypes = [C.c_int64, C.c_int, up32, C.c_uint64]
    lib.orc_nonempty_bins.restype = C.c_int64
    lib.orc_width_search.argtypes = [C.c_int64, C.c_int, up32, C.c_int64, up64, ip64,
                                     C.POINTER(C.c_int)]
    lib.orc_histogram.argtypes = [C.c_int64, C.c_int, up32, C.c_uint64, up64, ip64, i32p]
    lib.orc_histogram.restype = C.c_int64
    lib.orc_represent.argtypes = [C.c_int, C.c_int64, C.c_int, dp, C.c_int, dp, dp, dp,
                                  C.c_uint64, C.c_int64, up64, ip64, i32p, dp]
    lib.orc_bumbar.argtypes = [C.c_int, C.c_int64, dp, ip64, C.c_int, dp, C.c_int, dp,
                               C.c_int64, C.c_double, C.c_int64, C.c_int, C.c_double, C.c_int,
                               C.c_int64, C.c_int, C.POINTER(C.c_int), C.c_int, dp, dp,
                               C.POINTER(CheckRecord), C.c_int, ip64]
    lib.orc_reweight.argtypes = [C.c_int64, dp, dp, dp]
    lib.orc_pmf.argtypes = [C.c_int64, C.c_int, dp, dp, dp, dp, C.POINTER(C.c_int), dp]
    lib.orc_check_record_size.restype = C.c_int
    assert lib.orc_check_record_size() == C.sizeof(CheckRecord)
    _lib = lib
    return lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None else None


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def log_denominator(u, Nk, f):
    """ln D_n = LSE_{k: N_k>0}(ln N_k + f_k - u_kn): denominator of Eq. (1), Section 2."""
    u, Nk, f = _d(u), _i64(Nk), _d(f)
    K, P = u.shape
    out = np.empty(P)
    _check(_load().orc_log_denominator(K, P, _p(u), _p(Nk, C.c_int64), _p(f), _p(out)), "logD")
    return out


def sci_step(u, Nk, f, logH=None, return_logD=False):
    """One self-consistent iteration of Eq. (1) (Section 2), gauge f_0 = 0.

    ``u`` is K x P (bin representatives, or K x N samples when logH is None).
    """
    u, Nk, f = _d(u), _i64(Nk), _d(f)
    K, P = u.shape
    lh = _d(logH) if logH is not None else None
    fn = np.empty(K)
    ld = np.empty(P)
    _check(_load().orc_sci_step(K, P, _p(u), _p(lh), _p(Nk, C.c_int64), _p(f), _p(fn), _p(ld)),
           "sci")
    return (fn, ld) if return_logD else fn


def rel_step(f_new, f_old):
    """Relative step width, Eq. (2) (gauge state excluded)."""
    f_new, f_old = _d(f_new), _d(f_old)
    return float(_load().orc_rel_step(len(f_new), _p(f_new), _p(f_old)))


def weights(u, Nk, f):
    """W_nk = exp(f_k - u_kn - ln D_n), N x K."""
    u, Nk, f = _d(u), _i64(Nk), _d(f)
    K, N = u.shape
    W = np.empty((N, K))
    _check(_load().orc_weights(K, N, _p(u), _p(Nk, C.c_int64), _p(f), _p(W)), "weights")
    return W


def objective_gradient(u, Nk, f):
    """F(f) = sum_n ln D_n - sum_k N_k f_k and g_i = N_i (sum_n W_ni - 1)."""
    u, Nk, f = _d(u), _i64(Nk), _d(f)
    K, N = u.shape
    F = C.c_double()
    g = np.empty(K)
    _check(_load().orc_objective_gradient(K, N, _p(u), _p(Nk, C.c_int64), _p(f), C.byref(F),
                                          _p(g)), "objective")
    return F.value, g


def hessian(u, Nk, f):
    """H_ij = N_i d_ij sum_n W_ni - N_i N_j sum_n W_ni W_nj."""
    u, Nk, f = _d(u), _i64(Nk), _d(f)
    K, N = u.shape
    H = np.empty((K, K))
    _check(_load().orc_hessian(K, N, _p(u), _p(Nk, C.c_int64), _p(f), _p(H)), "hessian")
    return H


def newton_direction(Nk, H, g):
    Nk, H, g = _i64(Nk), _d(H), _d(g)
    d = np.empty(len(g))
    rc = _load().orc_newton_direction(len(g), _p(Nk, C.c_int64), _p(H), _p(g), _p(d))
    return d if rc == 0 else None


def newton_finish(u, Nk, f, tol=1e-12, max_steps=100):
    u, Nk = _d(u), _i64(Nk)
    f = _d(f).copy()
    K, N = u.shape
    st, fb = C.c_int(), C.c_int()
    rc = _load().orc_newton_finish(K, N, _p(u), _p(Nk, C.c_int64), _p(f), tol, max_steps,
                                   C.byref(st), C.byref(fb))
    return f, rc, st.value, fb.value


def solve_mbar(u, Nk, f_init=None, sci_switch=1e-3, sci_max=100000, newton_tol=1e-13,
               newton_max=60):
    """Certified unbinned MBAR solution: SCI, then the Newton finisher.

    Returns (f, info) with info = dict(rc, sci_steps, newton_steps, residual).
    """
    u, Nk = _d(u), _i64(Nk)
    K, N = u.shape
    fi = _d(f_init) if f_init is not None else None
    f = np.empty(K)
    s1, s2, res = C.c_int(), C.c_int(), C.c_double()
    rc = _load().orc_solve_mbar(K, N, _p(u), _p(Nk, C.c_int64), _p(fi), sci_switch, sci_max,
                                newton_tol, newton_max, _p(f), C.byref(s1), C.byref(s2),
                                C.byref(res))
    return f, dict(rc=rc, sci_steps=s1.value, newton_steps=s2.value, residual=res.value)


def quantize(xi):
    """Per-dimension 32-bit quantisation anchored at the minimum (binning, Section 2)."""
    xi = _d(xi)
    if xi.ndim == 1:
        xi = xi[:, None]
    N, d = xi.shape
    q = np.empty((N, d), dtype=np.uint32)
    lo, sc = np.empty(d), np.empty(d)
    _check(_load().orc_quantize(N, d, _p(xi), _p(q, C.c_uint32), _p(lo), _p(sc)), "quantize")
    return q, lo, sc


def nonempty_bins(q, m):
    q = np.ascontiguousarray(q, dtype=np.uint32)
    N, d = q.shape
    return int(_load().orc_nonempty_bins(N, d, _p(q, C.c_uint32), m))


def width_search(q, n_target):
    """w*(n) = max{w : n <= g(w)} by integer bisection (Section 2, after Eq. (1))."""
    q = np.ascontiguousarray(q, dtype=np.uint32)
    N, d = q.shape
    m, g, pr = C.c_uint64(), C.c_int64(), C.c_int()
    _check(_load().orc_width_search(N, d, _p(q, C.c_uint32), n_target, C.byref(m), C.byref(g),
                                    C.byref(pr)), "width_search")
    return m.value, g.value, pr.value


def histogram(q, m):
    """Nonempty bins (ascending cell id), counts H_p and the sample -> bin map."""
    q = np.ascontiguousarray(q, dtype=np.uint32)
    N, d = q.shape
    cells = np.empty(N, dtype=np.uint64)
    H = np.empty(N, dtype=np.int64)
    sb = np.empty(N, dtype=np.int32)
    P = _load().orc_histogram(N, d, _p(q, C.c_uint32), m, _p(cells, C.c_uint64),
                              _p(H, C.c_int64), _p(sb, C.c_int32))
    if P < 0:
        raise RuntimeError("oracle histogram failed")
    return cells[:P].copy(), H[:P].copy(), sb


def represent(K, d, m, lo, scale, cells, H, sample_bin=None, u=None, model_type=MODEL_NONE,
              coef=None):
    """Bin representatives ubar (K x P): model at the bin centre, or mean over members."""
    P = len(cells)
    cells = np.ascontiguousarray(cells, dtype=np.uint64)
    H = _i64(H)
    lo, scale = _d(lo), _d(scale)
    ub = np.empty((K, P))
    uu = _d(u) if u is not None else None
    N = uu.shape[1] if uu is not None else (len(sample_bin) if sample_bin is not None else 0)
    sb = np.ascontiguousarray(sample_bin, dtype=np.int32) if sample_bin is not None else None
    cf = _d(coef) if coef is not None else None
    _check(_load().orc_represent(K, N, d, _p(uu), model_type, _p(cf), _p(lo), _p(scale), m, P,
                                 _p(cells, C.c_uint64), _p(H, C.c_int64), _p(sb, C.c_int32),
                                 _p(ub)), "represent")
    return ub


def bumbar(u, Nk, xi, model_type=MODEL_NONE, coef=None, n0=100, eps=1e-3, inc=10, n_int=20,
           tol=1e-10, finisher=0, max_iter=2_000_000, replay=None):
    """Algorithm 1 (Section 2) followed by the unbinned finisher.

    ``replay`` = (phase1_steps, [refine flags]) replays a given schedule.
    Returns (f, info) with info = dict(rc, f_binned, checks (list of dicts), phase1, phase2,
    n_checks, finisher_steps).
    """
    u, Nk, xi = _d(u), _i64(Nk), _d(xi)
    if xi.ndim == 1:
        xi = xi[:, None]
    K, N = u.shape
    d = xi.shape[1]
    cf = _d(coef) if coef is not None else None
    f = np.empty(K)
    fb = np.empty(K)
    cap = 4096
    checks = (CheckRecord * cap)()
    counts = np.zeros(4, dtype=np.int64)
    rp1, rref, nrep = 0, None, 0
    if replay is not None:
        rp1 = int(replay[0])
        arr = (C.c_int * max(1, len(replay[1])))(*[int(x) for x in replay[1]])
        rref, nrep = arr, len(replay[1])
    rc = _load().orc_bumbar(K, N, _p(u), _p(Nk, C.c_int64), d, _p(xi), model_type, _p(cf), n0,
                            eps, inc, n_int, tol, finisher, max_iter, rp1, rref, nrep, _p(f),
                            _p(fb), checks, cap, _p(counts, C.c_int64))
    nck = int(counts[2])
    recs = [dict(n=c.n, P=c.P, P_next=c.P_next, s_n=c.s_n, s_next=c.s_next,
                 refine=c.refine, stop=c.stop) for c in checks[:min(nck, cap)]]
    return f, dict(rc=rc, f_binned=fb, checks=recs, phase1=int(counts[0]),
                   phase2=int(counts[1]), n_checks=nck, finisher_steps=int(counts[3]))


def reweight(u_target, logD):
    """Per-sample probabilities at a target state, Eqs. (5)-(6) (Section 3)."""
    ut, ld = _d(u_target), _d(logD)
    p = np.empty(len(ut))
    _check(_load().orc_reweight(len(ut), _p(ut), _p(ld), _p(p)), "reweight")
    return p


def pmf(xi, p, lo, hi, nbins):
    """Free-energy surface -ln sum_{n in bin} p_n on a regular grid (Section 3, Fig. 1)."""
    x = _d(xi)
    if x.ndim == 1:
        x = x[:, None]
    x = np.ascontiguousarray(x)
    N, d = x.shape
    lo_a, hi_a = _d(np.atleast_1d(lo)), _d(np.atleast_1d(hi))
    nb = np.ascontiguousarray(np.atleast_1d(nbins), dtype=np.int32)
    F = np.empty(int(np.prod(nb)))
    _check(_load().orc_pmf(N, d, _p(x), _p(_d(p)), _p(lo_a), _p(hi_a), _p(nb, C.c_int), _p(F)),
           "pmf")
    return F.reshape(tuple(int(v) for v in nb))


def covariance(u, Nk, f, null_tol=1e-9):
    """Asymptotic covariance of the free energies, Cov(f_i, f_j) in the gauge f_0 = 0.

    The paper names uncertainty estimates only as related work (Section 1);
    the estimator here is the large-sample covariance of the MBAR estimate
    (Shirts and Chodera, J. Chem. Phys. 129, 124105 (2008)):

        Theta = W^T (I_N - W diag(N_k) W^T)^+ W,   W_nk = exp(f_k - u_kn - ln D_n),

    at the solution f, and Cov(f_i, f_j) = (e_i - e_0)^T Theta (e_j - e_0).
    The N x N pseudo-inverse is written out through the thin SVD of
    A = W_S diag(N_S)^(1/2) over the sampled states S: with A = U diag(s) V^T,
    (I - A A^T)^+ = (I - U U^T) + U diag(h) U^T where h = 1 / (1 - s^2), and
    h = 0 on the null direction s = 1 (|1 - s^2| < null_tol; at the solution
    it is the gauge direction, A diag(N_S)^(1/2) 1 = 1_N). Returns K x K.
    """
    u, Nk, f = _d(u), _i64(Nk), _d(f)
    W = weights(u, Nk, f)
    S = Nk > 0
    A = W[:, S] * np.sqrt(Nk[S].astype(np.float64))
    U, s, _ = np.linalg.svd(A, full_matrices=False)
    gap = 1.0 - s * s
    h = np.where(np.abs(gap) < null_tol, 0.0, 1.0 / np.where(np.abs(gap) < null_tol, 1.0, gap))
    WU = W.T @ U
    theta = W.T @ W - WU @ WU.T + (WU * h) @ WU.T
    return theta - theta[:, :1] - theta[:1, :] + theta[0, 0]
