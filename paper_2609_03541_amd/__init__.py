"""MI355X (gfx950) BU-MBAR solver: Python binding of libbumbar.so.

The binding only marshals arguments. PyTorch supplies device memory and the
HIP stream: pass CUDA (HIP) tensors, results come back as tensors on the same
device. Every step of the solve runs in the HIP kernels of libbumbar.

    import torch, paper_2609_03541_amd as bm
    f, info = bm.solve(u_kn, N_k, xi=xi, model=bm.MODEL_HARMONIC, coef=coef, binning=True)
"""
from __future__ import annotations

import ctypes as C

from . import _capi
from ._capi import (EBUSY, EDEVICE, EINVAL, ENOMEM, ENOTCONV, ETOOBIG, F32, F64,  # noqa: F401
                    FINISH_NEWTON, FINISH_SCI, MODEL_HARMONIC, MODEL_LINEAR, MODEL_NONE, OK,
                    PREC_FP64, PREC_MIXED, REPRESENT_AUTO, REPRESENT_CENTRE, REPRESENT_MEAN)

__all__ = ["Context", "solve", "plan", "sweep", "sample_major", "SampleMajor", "hessian", "weights", "bin_coordinates", "reweight", "pmf",
           "model_energies", "sweep_model", "hessian_model", "Server", "covariance",
           "BumbarError", "default_options"]


class BumbarError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bumbar error {code}: {msg}")
        self.code = code


def _torch():
    import torch
    return torch


class Context:
    """A library context bound to one device and one HIP stream."""

    def __init__(self, device=None, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libbumbar needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = _capi.load()
        dev = torch.cuda.current_device() if device is None else int(device)
        self.device = dev
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        self.stream = st
        h = C.c_void_p()
        rc = self.lib.bumbar_create(C.byref(h), dev, C.c_void_p(st.cuda_stream))
        if rc != 0:
            raise BumbarError(rc, "bumbar_create failed")
        self.h = h
        self._ws = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.bumbar_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self):
        return self.lib.bumbar_last_error(self.h).decode()

    def check(self, rc, allow=()):
        if rc != 0 and rc not in allow:
            raise BumbarError(rc, self.error())
        return rc

    def workspace(self, nbytes):
        torch = _torch()
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def query_workspace(self, K, N, d=0, opts=None):
        nb = C.c_size_t()
        o = C.byref(opts) if opts is not None else None
        self.check(self.lib.bumbar_query_workspace(self.h, K, N, d, o, C.byref(nb)))
        return nb.value

    def step_workspace(self, K, N):
        """Workspace of the single-step calls (no binning, no sample-major copy)."""
        return self.query_workspace(K, N, 0, default_options(sample_major=0))


_default_ctx = {}


def context(device=None):
    torch = _torch()
    dev = torch.cuda.current_device() if device is None else int(device)
    key = (dev, torch.cuda.current_stream(dev).cuda_stream)
    if key not in _default_ctx:
        _default_ctx[key] = Context(dev)
    return _default_ctx[key]


def plan(K, N, d=0, model=MODEL_NONE, u_dtype=F64, stored_u=True, num_cus=256, **options):
    """What bumbar_solve would run for this shape and options (bumbar_plan_solve, host only).

    Raises BumbarError for a combination the solver refuses."""
    lib = _capi.load()
    o = default_options(**options)
    p = _capi.Plan()
    msg = C.create_string_buffer(256)
    rc = lib.bumbar_plan_solve(num_cus, int(bool(stored_u)), u_dtype, K, N, d, model, C.byref(o),
                               C.byref(p), msg, 256)
    if rc != 0:
        raise BumbarError(rc, msg.value.decode())
    return {f: getattr(p, f) for f, _ in _capi.Plan._fields_}


def default_options(**kw):
    o = _capi.Options()
    _capi.load().bumbar_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        if k == "trace_path" and isinstance(v, str):
            v = v.encode()
        setattr(o, k, v)
    return o


def _keep(ctx, *tensors):
    """Hold the temporaries of an asynchronous call until the stream passes this point.

    The library queues kernels and returns; a tensor created only to pass a
    pointer must not go back to the caching allocator before those kernels
    run. record_stream ties the block to the context's stream.
    """
    for t in tensors:
        if t is not None:
            t.record_stream(ctx.stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, device):
    torch = _torch()
    if t is None:
        return None
    if not torch.is_tensor(t):
        t = torch.as_tensor(t)
    return t.to(device=device, dtype=dtype).contiguous()


def _dtype_code(u):
    torch = _torch()
    if u.dtype == torch.float64:
        return F64
    if u.dtype == torch.float32:
        return F32
    raise TypeError("u_kn and xi must be float64 or float32")


def _is_f32(a):
    import numpy as np
    torch = _torch()
    if torch.is_tensor(a):
        return a.dtype == torch.float32
    return getattr(a, "dtype", None) == np.float32


def solve(u, Nk, xi=None, model=MODEL_NONE, coef=None, f_init=None, binning=None,
          want_weights=False, want_logD=False, ctx=None, checks_capacity=256, **options):
    """Solve the MBAR equations for u (K x N) and counts Nk (K).

    ``u = None`` takes the energies from the model (``xi``, ``model``,
    ``coef`` required): they are evaluated inside the kernels, never stored.
    ``binning`` defaults to True when coordinates ``xi`` (N x d) are given.
    Keyword options are the fields of ``bumbar_options`` (tol, precision,
    n0, eps, inc, n_intermediate, finisher, max_iter, max_newton, sci_switch).
    ``replay=(phase1_steps, [refine flags])`` replays a phase-2 schedule.
    Returns (f, info): f is a float64 tensor on the device; info holds the
    statistics, the phase-2 schedule and optional W (N x K) and ln D (N).
    """
    torch = _torch()
    ctx = ctx or context()
    dev = torch.device(f"cuda:{ctx.device}")
    if u is not None:
        if not (torch.is_tensor(u) and u.is_cuda):
            u = torch.as_tensor(u)
        u = u.to(dev).contiguous()
        K, N = u.shape
    Nk_t = _dev(Nk, torch.int64, dev)
    d = 0
    xi_t = None
    if xi is not None:
        # FP32 coordinates travel as FP32 (the library widens them exactly)
        xi_t = _dev(xi, torch.float32 if _is_f32(xi) else torch.float64, dev)
        if xi_t.dim() == 1:
            xi_t = xi_t[:, None].contiguous()
        d = xi_t.shape[1]
        options.setdefault("xi_dtype", _dtype_code(xi_t))
    if u is None:
        # energies from the model, evaluated inside the kernels
        if xi_t is None or coef is None or model == MODEL_NONE:
            raise ValueError("u = None needs xi, a model and its coefficients")
        K, N = Nk_t.numel(), xi_t.shape[0]
    if binning is None:
        binning = xi is not None
    replay = options.pop("replay", None)
    options.setdefault("represent", _capi.REPRESENT_CENTRE if model != MODEL_NONE
                       else _capi.REPRESENT_MEAN)
    if u is not None:
        options.setdefault("u_dtype", _dtype_code(u))
    opts = default_options(binning=int(bool(binning)), **options)
    keep = None
    if replay is not None:
        arr = (C.c_int * max(1, len(replay[1])))(*[int(x) for x in replay[1]])
        keep = arr
        opts.replay_phase1 = int(replay[0])
        opts.replay_refine = C.cast(arr, C.POINTER(C.c_int))
        opts.n_replay = len(replay[1])
    coef_t = _dev(coef, torch.float64, dev) if coef is not None else None
    f_init_t = _dev(f_init, torch.float64, dev) if f_init is not None else None
    if u is None:
        nb = C.c_size_t()
        ctx.check(ctx.lib.bumbar_query_workspace_model(ctx.h, K, N, d, C.byref(opts),
                                                       C.byref(nb)))
        nbytes = nb.value
    else:
        nbytes = ctx.query_workspace(K, N, d if binning else 0, opts)
    ws = ctx.workspace(nbytes)
    f = torch.empty(K, dtype=torch.float64, device=dev)
    W = torch.empty((N, K), dtype=torch.float64, device=dev) if want_weights else None
    lD = torch.empty(N, dtype=torch.float64, device=dev) if want_logD else None
    st = _capi.Stats()
    chk = (_capi.Check * max(1, checks_capacity))()
    st.checks = C.cast(chk, C.POINTER(_capi.Check))
    st.checks_capacity = checks_capacity
    rc = ctx.lib.bumbar_solve(ctx.h, _ptr(u), _dtype_code(u) if u is not None else F64, K, N,
                              _ptr(Nk_t), _ptr(xi_t),
                              _dtype_code(xi_t) if xi_t is not None else F64, d, int(model),
                              _ptr(coef_t), _ptr(f_init_t), C.byref(opts), _ptr(ws), ws.numel(),
                              _ptr(f), _ptr(W), _ptr(lD), C.byref(st))
    del keep
    _keep(ctx, Nk_t, xi_t, coef_t, f_init_t, u)
    ctx.check(rc, allow=(ENOTCONV,))
    info = {name: getattr(st, name) for name, _ in _capi.Stats._fields_
            if name not in ("checks", "checks_capacity")}
    info["status"] = rc
    n = min(int(st.n_checks), checks_capacity)
    info["checks"] = [dict(n=c.n, P=c.P, P_next=c.P_next, s_n=c.s_n, s_next=c.s_next,
                           refine=c.refine, stop=c.stop) for c in chk[:n]]
    if W is not None:
        info["W"] = W
    if lD is not None:
        info["logD"] = lD
    return f, info


class SampleMajor:
    """The sample-major copy of a K x N matrix (``sample_major``): device data plus its shape."""

    def __init__(self, data, K, N, code):
        self.data, self.K, self.N, self.code = data, K, N, code
        self.device = data.device
        self.shape = (K, N)


def sample_major(u, ctx=None):
    """Sample-major copy of u (K x N state-major, 256 < K <= 1024) for ``sweep``."""
    torch = _torch()
    ctx = ctx or context()
    K, N = u.shape
    code = _dtype_code(u)
    n = ctx.lib.bumbar_sample_major_elems(K, N)
    if n < 0:
        raise BumbarError(EINVAL, "the sample-major layout is defined for 256 < K <= 1024")
    out = torch.empty(int(n), dtype=u.dtype, device=u.device)
    ctx.check(ctx.lib.bumbar_sample_major(ctx.h, _ptr(u), code, K, N, u.stride(0), _ptr(out)))
    _keep(ctx, u)
    return SampleMajor(out, K, N, _capi.F64_SMAJOR if code == F64 else _capi.F32_SMAJOR)


def sweep(u, Nk, f, ld=None, ctx=None, with_stats=True, want_logD=True):
    """One unbinned SCI step (Eq. (1), one sample per bin). Returns f_new, ln D, S, stats.

    ``u`` is a K x N tensor or the ``SampleMajor`` copy of one. With
    ``want_logD=False`` no ln D is written (the form the SCI iteration uses)
    and None is returned in its place."""
    torch = _torch()
    ctx = ctx or context()
    dev = u.device
    K, N = u.shape[0], u.shape[1]
    if isinstance(u, SampleMajor):
        code, ld, uptr = u.code, N, _ptr(u.data)
    else:
        code, ld, uptr = _dtype_code(u), (u.stride(0) if ld is None else ld), _ptr(u)
    Nk_t = _dev(Nk, torch.int64, dev)
    f_t = _dev(f, torch.float64, dev)
    ws = ctx.workspace(ctx.step_workspace(K, N))
    f_new = torch.empty(K, dtype=torch.float64, device=dev)
    lD = torch.empty(N, dtype=torch.float64, device=dev) if want_logD else None
    S = torch.empty(K, dtype=torch.float64, device=dev)
    stats = (C.c_double * 4)() if with_stats else None
    rc = ctx.lib.bumbar_sweep(ctx.h, uptr, code, K, N, ld, _ptr(Nk_t), _ptr(f_t),
                              _ptr(ws), ws.numel(), _ptr(f_new),
                              _ptr(lD), _ptr(S),
                              C.cast(stats, C.POINTER(C.c_double)) if stats else None)
    ctx.check(rc)
    _keep(ctx, Nk_t, f_t)
    st = None
    if stats is not None:
        st = dict(max_df=stats[0], rel_step=stats[1], objective=stats[2], grad_norm=stats[3])
    return f_new, lD, S, st


def hessian(u, Nk, f, logD, S, ctx=None, fp16=False):
    """K x K Hessian of the MBAR objective at f (FP64 MFMA; fp16=True: the
    FP16-core Hessian of the K > 256 Newton steps)."""
    torch = _torch()
    ctx = ctx or context()
    dev = u.device
    K, N = u.shape
    ws = ctx.workspace(ctx.step_workspace(K, N))
    H = torch.empty((K, K), dtype=torch.float64, device=dev)
    # keep every marshalled tensor alive until the queued kernels have run
    Nk_t = _dev(Nk, torch.int64, dev)
    f_t = _dev(f, torch.float64, dev)
    fn = ctx.lib.bumbar_hessian_fp16 if fp16 else ctx.lib.bumbar_hessian
    rc = fn(ctx.h, _ptr(u), _dtype_code(u), K, N, u.stride(0), _ptr(Nk_t), _ptr(f_t),
            _ptr(logD), _ptr(S), _ptr(ws), ws.numel(), _ptr(H))
    ctx.check(rc)
    _keep(ctx, Nk_t, f_t)
    return H


def covariance(u, Nk, f, ctx=None):
    """K x K asymptotic covariance of f at the solution f (gauge f_0 = 0), on the device."""
    torch = _torch()
    ctx = ctx or context()
    if not (torch.is_tensor(u) and u.is_cuda):
        u = torch.as_tensor(u)
    dev = torch.device(f"cuda:{ctx.device}")
    u = u.to(dev)
    if u.stride(1) != 1:
        u = u.contiguous()
    K, N = u.shape
    nb = C.c_size_t()
    ctx.check(ctx.lib.bumbar_query_workspace_covariance(ctx.h, K, N, C.byref(nb)))
    ws = ctx.workspace(nb.value)
    cov = torch.empty((K, K), dtype=torch.float64, device=dev)
    Nk_t = _dev(Nk, torch.int64, dev)
    f_t = _dev(f, torch.float64, dev)
    rc = ctx.lib.bumbar_covariance(ctx.h, _ptr(u), _dtype_code(u), K, N, u.stride(0), _ptr(Nk_t),
                                   _ptr(f_t), _ptr(ws), ws.numel(), _ptr(cov))
    _keep(ctx, Nk_t, f_t, u)
    ctx.check(rc)
    return cov


def weights(u, f, logD, ctx=None):
    """W_nk = exp(f_k - u_kn - ln D_n), N x K."""
    torch = _torch()
    ctx = ctx or context()
    K, N = u.shape
    W = torch.empty((N, K), dtype=torch.float64, device=u.device)
    f_t = _dev(f, torch.float64, u.device)
    rc = ctx.lib.bumbar_weights(ctx.h, _ptr(u), _dtype_code(u), K, N, u.stride(0), _ptr(f_t),
                                _ptr(logD), _ptr(W))
    ctx.check(rc)
    _keep(ctx, f_t)
    return W


def bin_coordinates(xi, n_target, ctx=None):
    """Width search and histogram for a target of n nonempty bins.

    Returns (m, cells (P, uint64 as int64 tensor), H (P), sample_bin (N)).
    """
    torch = _torch()
    ctx = ctx or context()
    dev = torch.device(f"cuda:{ctx.device}")
    xi_t = _dev(xi, torch.float64, dev)
    if xi_t.dim() == 1:
        xi_t = xi_t[:, None].contiguous()
    N, d = xi_t.shape
    ws = ctx.workspace(ctx.query_workspace(1, N, d))
    cells = torch.empty(N, dtype=torch.int64, device=dev)
    H = torch.empty(N, dtype=torch.int64, device=dev)
    sb = torch.empty(N, dtype=torch.int32, device=dev)
    m = C.c_uint64()
    P = C.c_int64()
    rc = ctx.lib.bumbar_bin(ctx.h, _ptr(xi_t), N, d, int(n_target), _ptr(ws), ws.numel(),
                            C.byref(m), C.byref(P), _ptr(cells), _ptr(H), _ptr(sb))
    ctx.check(rc)
    return m.value, cells[:P.value], H[:P.value], sb


def reweight(u_target, logD, ctx=None):
    """Per-sample probabilities at a target state (Eqs. (5)-(6))."""
    torch = _torch()
    ctx = ctx or context()
    N = u_target.numel()
    ws = ctx.workspace(8 * (2 * 1024 + 2))
    p = torch.empty(N, dtype=torch.float64, device=u_target.device)
    rc = ctx.lib.bumbar_reweight(ctx.h, _ptr(u_target), N, _ptr(logD), _ptr(ws), ws.numel(),
                                 _ptr(p))
    ctx.check(rc)
    return p


def pmf(xi, p, lo, hi, nbins, ctx=None):
    """Free-energy surface F_b = -ln sum_{n in bin b} p_n on a regular grid.

    xi: N x d coordinates (d in {1, 2}), p: N probabilities (from ``reweight``),
    lo, hi, nbins: d values each. Returns F as a float64 tensor of shape
    ``nbins`` (+inf for bins without probability).
    """
    torch = _torch()
    ctx = ctx or context()
    dev = torch.device(f"cuda:{ctx.device}")
    xi_t = _dev(xi, torch.float64, dev)
    if xi_t.dim() == 1:
        xi_t = xi_t[:, None].contiguous()
    N, d = xi_t.shape
    p_t = _dev(p, torch.float64, dev)

    def seq(v):
        return [v] if not hasattr(v, "__len__") else list(v)

    lo_l, hi_l, nb = [float(v) for v in seq(lo)], [float(v) for v in seq(hi)], \
        [int(v) for v in seq(nbins)]
    if not (len(lo_l) == len(hi_l) == len(nb) == d):
        raise ValueError("lo, hi and nbins need one entry per coordinate")
    lo_a, hi_a, nb_a = (C.c_double * d)(*lo_l), (C.c_double * d)(*hi_l), (C.c_int * d)(*nb)
    nbytes = C.c_size_t()
    ctx.check(ctx.lib.bumbar_query_workspace_pmf(ctx.h, N, C.byref(nbytes)))
    ws = ctx.workspace(nbytes.value)
    total = 1
    for v in nb:
        total *= v
    F = torch.empty(total, dtype=torch.float64, device=dev)
    rc = ctx.lib.bumbar_pmf(ctx.h, _ptr(xi_t), N, d, _ptr(p_t), lo_a, hi_a, nb_a, _ptr(ws),
                            ws.numel(), _ptr(F))
    _keep(ctx, xi_t, p_t)
    ctx.check(rc)
    return F.reshape(nb)


def _model_args(xi, coef, ctx):
    torch = _torch()
    dev = torch.device(f"cuda:{ctx.device}")
    xi_t = _dev(xi, torch.float64, dev)
    if xi_t.dim() == 1:
        xi_t = xi_t[:, None].contiguous()
    return xi_t, _dev(coef, torch.float64, dev)


def _model_ws(ctx, K, N, d):
    nb = C.c_size_t()
    ctx.check(ctx.lib.bumbar_query_workspace_model(ctx.h, K, N, d, None, C.byref(nb)))
    return ctx.workspace(nb.value)


def sweep_model(xi, coef, model, Nk, f, precision=PREC_FP64, ctx=None):
    """One unbinned SCI step with u from the model (FP64, or FP32 with precision=PREC_MIXED).

    Returns f_new, ln D, S and the scalars (max_df, rel_step, objective, grad_norm)."""
    torch = _torch()
    ctx = ctx or context()
    xi_t, coef_t = _model_args(xi, coef, ctx)
    N, d = xi_t.shape
    dev = xi_t.device
    Nk_t = _dev(Nk, torch.int64, dev)
    K = Nk_t.numel()
    f_t = _dev(f, torch.float64, dev)
    ws = _model_ws(ctx, K, N, d)
    f_new = torch.empty(K, dtype=torch.float64, device=dev)
    lD = torch.empty(N, dtype=torch.float64, device=dev)
    S = torch.empty(K, dtype=torch.float64, device=dev)
    stats = (C.c_double * 4)()
    rc = ctx.lib.bumbar_sweep_model(ctx.h, K, N, d, int(model), _ptr(coef_t), _ptr(xi_t),
                                    int(precision), _ptr(Nk_t), _ptr(f_t), _ptr(ws), ws.numel(),
                                    _ptr(f_new), _ptr(lD), _ptr(S), stats)
    _keep(ctx, xi_t, coef_t, Nk_t, f_t)
    ctx.check(rc)
    return f_new, lD, S, dict(max_df=stats[0], rel_step=stats[1], objective=stats[2],
                              grad_norm=stats[3])


def hessian_model(xi, coef, model, Nk, f, logD, S, precision=PREC_FP64, ctx=None):
    """K x K Hessian of the MBAR objective with u from the model."""
    torch = _torch()
    ctx = ctx or context()
    xi_t, coef_t = _model_args(xi, coef, ctx)
    N, d = xi_t.shape
    dev = xi_t.device
    Nk_t = _dev(Nk, torch.int64, dev)
    K = Nk_t.numel()
    f_t = _dev(f, torch.float64, dev)
    lD_t = _dev(logD, torch.float64, dev)
    S_t = _dev(S, torch.float64, dev)
    ws = _model_ws(ctx, K, N, d)
    H = torch.empty((K, K), dtype=torch.float64, device=dev)
    rc = ctx.lib.bumbar_hessian_model(ctx.h, K, N, d, int(model), _ptr(coef_t), _ptr(xi_t),
                                      int(precision), _ptr(Nk_t), _ptr(f_t), _ptr(lD_t),
                                      _ptr(S_t), _ptr(ws), ws.numel(), _ptr(H))
    _keep(ctx, xi_t, coef_t, Nk_t, f_t, lD_t, S_t)
    ctx.check(rc)
    return H


def model_energies(xi, coef, model, K, ctx=None, dtype=None):
    """u_kn = model_k(xi_n) (K x N) built on the device from coordinates xi (N x d).

    Evaluated in FP64; ``dtype=torch.float32`` stores it rounded to FP32."""
    torch = _torch()
    dtype = torch.float64 if dtype is None else dtype
    ctx = ctx or context()
    dev = torch.device(f"cuda:{ctx.device}")
    xi_t = _dev(xi, torch.float64, dev)
    if xi_t.dim() == 1:
        xi_t = xi_t[:, None].contiguous()
    N, d = xi_t.shape
    coef_t = _dev(coef, torch.float64, dev)
    u = torch.empty((K, N), dtype=dtype, device=dev)
    rc = ctx.lib.bumbar_model_energies(ctx.h, int(K), int(N), int(d), int(model), _ptr(coef_t),
                                       _ptr(xi_t), _dtype_code(u), _ptr(u))
    _keep(ctx, xi_t, coef_t)
    ctx.check(rc)
    return u


class Server:
    """Continuous batching of independent solves on one device.

    ``submit`` takes host (numpy) arrays and returns a ticket; the server
    admits requests in arrival order whenever a slot is free and the problem
    fits in the device arena of ``hbm_budget_bytes`` reserved at creation.
    The arrays are held here until the ticket's result has been read.
    """

    def __init__(self, hbm_budget_bytes, max_active=4, device=None, caller_driven=False,
                 fuse=False):
        import numpy  # noqa: F401  (requests are host arrays)
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("libbumbar needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = _capi.load()
        dev = torch.cuda.current_device() if device is None else int(device)
        o = _capi.ServerOptions(dev, int(hbm_budget_bytes), int(max_active), int(caller_driven),
                                int(bool(fuse)))
        self.caller_driven = bool(caller_driven)
        h = C.c_void_p()
        rc = self.lib.bumbar_server_create(C.byref(o), C.byref(h))
        if rc != 0:
            raise BumbarError(rc, "bumbar_server_create failed")
        self.h = h
        self._held = {}

    def submit(self, Nk, u=None, xi=None, model=MODEL_NONE, coef=None, K=None, binning=None,
               materialize=False, u_dtype=None, **options):
        """Queue one problem. Give u (K x N host array, float64 or float32), or
        xi + model + coef: the energies are then evaluated inside the kernels, or,
        with ``materialize=True``, once into a resident device u of ``u_dtype``
        (numpy.float32 by default) that the solve reads as a stored matrix.
        float32 coordinates travel as float32."""
        import numpy as np
        if "replay" in options:
            raise ValueError("replayed schedules are not supported by the server")
        if u is None and (xi is None or coef is None or model == MODEL_NONE):
            raise ValueError("give u, or xi with a model and its coefficients")
        arrs = {}
        udt = F64
        if u is not None:
            f32 = getattr(u, "dtype", None) == np.float32
            arrs["u"] = np.ascontiguousarray(u, dtype=np.float32 if f32 else np.float64)
            udt = F32 if f32 else F64
            K, N = arrs["u"].shape
        elif materialize:
            udt = F64 if u_dtype in (np.float64, F64) else F32
        arrs["Nk"] = np.ascontiguousarray(Nk, dtype=np.int64)
        K = int(K if K is not None else arrs["Nk"].shape[0])
        d = 0
        xdt = F64
        if xi is not None:
            f32 = getattr(xi, "dtype", None) == np.float32
            x = np.ascontiguousarray(xi, dtype=np.float32 if f32 else np.float64)
            if x.ndim == 1:
                x = x[:, None]
            arrs["xi"] = x
            xdt = F32 if f32 else F64
            N, d = x.shape
        if coef is not None:
            arrs["coef"] = np.ascontiguousarray(coef, dtype=np.float64)
        if binning is None:
            binning = xi is not None
        req = _capi.Request()
        req.K, req.N, req.d, req.model = K, int(N), int(d), int(model)
        req.u_dtype, req.xi_dtype, req.materialize = udt, xdt, int(bool(materialize))

        def p(name):
            a = arrs.get(name)
            return C.c_void_p(a.ctypes.data) if a is not None else None

        req.u_kn, req.N_k, req.xi, req.coef = p("u"), p("Nk"), p("xi"), p("coef")
        options.setdefault("represent", _capi.REPRESENT_CENTRE if model != MODEL_NONE
                           else _capi.REPRESENT_MEAN)
        options.setdefault("u_dtype", udt)
        options.setdefault("xi_dtype", xdt)
        req.opt = default_options(binning=int(bool(binning)), **options)
        t = C.c_uint64()
        rc = self.lib.bumbar_server_submit(self.h, C.byref(req), C.byref(t))
        if rc != 0:
            raise BumbarError(rc, "bumbar_server_submit failed")
        self._held[t.value] = (arrs, K)
        return t.value

    def poll(self, ticket):
        s = C.c_int()
        rc = self.lib.bumbar_server_poll(self.h, C.c_uint64(ticket), C.byref(s))
        if rc != 0:
            raise BumbarError(rc, "unknown ticket")
        return s.value

    def wait(self, ticket):
        rc = self.lib.bumbar_server_wait(self.h, C.c_uint64(ticket))
        if rc != 0:
            raise BumbarError(rc, "unknown ticket")

    def progress(self):
        """One tick of a caller-driven server; returns the number of tickets it finished."""
        n = C.c_int()
        rc = self.lib.bumbar_server_progress(self.h, C.byref(n))
        if rc != 0:
            raise BumbarError(rc, "bumbar_server_progress failed")
        return n.value

    def result(self, ticket, wait=True):
        """(f as numpy float64, info) of a finished ticket; waits for it by default.

        The ticket is released once its result has been read."""
        import numpy as np
        if wait:
            self.wait(ticket)
        _, K = self._held[ticket]
        f = np.empty(K, dtype=np.float64)
        st = _capi.Stats()
        lat = C.c_double()
        status = C.c_int()
        rc = self.lib.bumbar_server_result(self.h, C.c_uint64(ticket), C.c_void_p(f.ctypes.data),
                                           C.byref(st), C.byref(lat), C.byref(status))
        if rc != 0:
            raise BumbarError(rc, "result not available")
        info = {name: getattr(st, name) for name, _ in _capi.Stats._fields_
                if name not in ("checks", "checks_capacity")}
        info["latency_ms"] = lat.value
        info["status"] = status.value
        del self._held[ticket]
        return f, info

    def counters(self):
        c, a, b, w = C.c_int64(), C.c_int64(), C.c_size_t(), C.c_int64()
        self.lib.bumbar_server_counters(self.h, C.byref(c), C.byref(a), C.byref(b), C.byref(w))
        fl, fi = C.c_int64(), C.c_int64()
        self.lib.bumbar_server_fused_counters(self.h, C.byref(fl), C.byref(fi))
        return dict(completed=c.value, peak_active=a.value, peak_bytes=b.value,
                    mem_waits=w.value, fused_launches=fl.value, fused_items=fi.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.bumbar_server_destroy(self.h)
            self.h = None
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
