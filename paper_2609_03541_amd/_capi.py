"""ctypes declarations of libbumbar.so (the C ABI in include/bumbar.h).

Argument marshalling only: every computation runs in the HIP library. The
library is loaded from this package directory; if it has not been built the
import of the binding fails loudly (there is no fallback implementation).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbumbar.so")

OK = 0
EINVAL = -1
ENOMEM = -2
EDEVICE = -3
ENOTCONV = -4
ETOOBIG = -5
EBUSY = -6

F64 = 0
F32 = 1
F64_SMAJOR = 2
F32_SMAJOR = 3
PREC_FP64 = 0
PREC_MIXED = 1
FINISH_NEWTON = 0
FINISH_SCI = 1
MODEL_NONE = 0
MODEL_LINEAR = 1
MODEL_HARMONIC = 2
REPRESENT_AUTO = 0
REPRESENT_CENTRE = 1
REPRESENT_MEAN = 2
TICKET_QUEUED = 0
TICKET_RUNNING = 1
TICKET_DONE = 2
TICKET_FAILED = 3


class Check(C.Structure):
    _fields_ = [("n", C.c_int64), ("P", C.c_int64), ("P_next", C.c_int64),
                ("s_n", C.c_double), ("s_next", C.c_double), ("refine", C.c_int),
                ("stop", C.c_int)]


class Options(C.Structure):
    _fields_ = [("tol", C.c_double), ("precision", C.c_int), ("binning", C.c_int),
                ("n0", C.c_int64), ("eps", C.c_double), ("inc", C.c_int64),
                ("n_intermediate", C.c_int), ("finisher", C.c_int), ("max_iter", C.c_int64),
                ("max_newton", C.c_int), ("sci_switch", C.c_double),
                ("replay_phase1", C.c_int), ("replay_refine", C.POINTER(C.c_int)),
                ("n_replay", C.c_int), ("profile", C.c_int), ("mixed_tol", C.c_double),
                ("represent", C.c_int), ("graphs", C.c_int), ("sample_major", C.c_int),
                ("u_dtype", C.c_int), ("xi_dtype", C.c_int), ("trace_path", C.c_char_p),
                ("grid_batches", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("phase1_iters", C.c_int64), ("phase2_iters", C.c_int64),
                ("n_checks", C.c_int64), ("finisher_steps", C.c_int64),
                ("sci_fallbacks", C.c_int64), ("unbinned_sweeps", C.c_int64),
                ("robust_sweeps", C.c_int64), ("hessians", C.c_int64),
                ("mixed_steps", C.c_int64),
                ("final_step", C.c_double), ("grad_norm", C.c_double),
                ("time_binning_ms", C.c_double), ("time_binned_ms", C.c_double),
                ("time_final_ms", C.c_double), ("sweep_kernel_ms", C.c_double),
                ("sweep_kernel_launches", C.c_int64), ("checks", C.POINTER(Check)),
                ("checks_capacity", C.c_int), ("graph_batches", C.c_int64),
                ("grid_sweeps", C.c_int64), ("batched_steps", C.c_int64),
                ("damped_steps", C.c_int64), ("coop_steps", C.c_int64)]


class Plan(C.Structure):
    _fields_ = [("precision", C.c_int), ("represent", C.c_int), ("sweep", C.c_int),
                ("stage32", C.c_int), ("fp32_binned", C.c_int), ("hessian_fp16", C.c_int),
                ("copy_bytes", C.c_size_t), ("workspace_bytes", C.c_size_t)]


SWEEP_REGISTER = 0
SWEEP_SAMPLE_MAJOR = 1
SWEEP_TWO_PASS = 2
SWEEP_MODEL = 3
STAGE32_NONE = 0
STAGE32_PACKED = 1
STAGE32_SAMPLE_MAJOR = 2
STAGE32_MODEL = 3
STAGE32_STORED = 4


class ServerOptions(C.Structure):
    _fields_ = [("device", C.c_int), ("hbm_budget_bytes", C.c_size_t), ("max_active", C.c_int),
                ("caller_driven", C.c_int), ("fuse", C.c_int)]


class Request(C.Structure):
    _fields_ = [("K", C.c_int), ("N", C.c_int64), ("u_kn", C.c_void_p), ("u_dtype", C.c_int),
                ("N_k", C.c_void_p), ("xi", C.c_void_p), ("xi_dtype", C.c_int),
                ("d", C.c_int), ("model", C.c_int), ("coef", C.c_void_p),
                ("materialize", C.c_int), ("opt", Options)]


# name -> (restype, argtypes); the full exported surface of include/bumbar.h
vp, dp, i64p, u64p, i32p = (C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                            C.POINTER(C.c_uint64), C.POINTER(C.c_int32))
SIGNATURES = {
    "bumbar_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, vp]),
    "bumbar_destroy": (None, [vp]),
    "bumbar_last_error": (C.c_char_p, [vp]),
    "bumbar_version": (C.c_char_p, []),
    "bumbar_default_options": (None, [C.POINTER(Options)]),
    "bumbar_query_workspace": (C.c_int, [vp, C.c_int, C.c_int64, C.c_int, C.POINTER(Options),
                                         C.POINTER(C.c_size_t)]),
    "bumbar_plan_solve": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, C.c_int,
                                    C.c_int, C.POINTER(Options), C.POINTER(Plan), C.c_char_p,
                                    C.c_size_t]),
    "bumbar_solve": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_int64, vp, vp, C.c_int, C.c_int,
                               C.c_int, vp, vp, C.POINTER(Options), vp, C.c_size_t, vp, vp, vp,
                               C.POINTER(Stats)]),
    "bumbar_sweep": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_int64, C.c_int64, vp, vp, vp,
                               C.c_size_t, vp, vp, vp, dp]),
    "bumbar_hessian": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_int64, C.c_int64, vp, vp, vp, vp,
                                 vp, C.c_size_t, vp]),
    "bumbar_hessian_fp16": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_int64, C.c_int64, vp, vp, vp,
                                      vp, vp, C.c_size_t, vp]),
    "bumbar_query_workspace_covariance": (C.c_int, [vp, C.c_int, C.c_int64,
                                                    C.POINTER(C.c_size_t)]),
    "bumbar_covariance": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_int64, C.c_int64, vp, vp, vp,
                                    C.c_size_t, vp]),
    "bumbar_sample_major_elems": (C.c_int64, [C.c_int, C.c_int64]),
    "bumbar_sample_major": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_int64, C.c_int64, vp]),
    "bumbar_weights": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_int64, C.c_int64, vp, vp, vp]),
    "bumbar_bin": (C.c_int, [vp, vp, C.c_int64, C.c_int, C.c_int64, vp, C.c_size_t, u64p, i64p,
                             vp, vp, vp]),
    "bumbar_reweight": (C.c_int, [vp, vp, C.c_int64, vp, vp, C.c_size_t, vp]),
    "bumbar_query_workspace_pmf": (C.c_int, [vp, C.c_int64, C.POINTER(C.c_size_t)]),
    "bumbar_pmf": (C.c_int, [vp, vp, C.c_int64, C.c_int, vp, dp, dp, C.POINTER(C.c_int), vp,
                             C.c_size_t, vp]),
    "bumbar_query_workspace_model": (C.c_int, [vp, C.c_int, C.c_int64, C.c_int,
                                               C.POINTER(Options), C.POINTER(C.c_size_t)]),
    "bumbar_sweep_model": (C.c_int, [vp, C.c_int, C.c_int64, C.c_int, C.c_int, vp, vp, C.c_int, vp,
                                     vp, vp, C.c_size_t, vp, vp, vp, dp]),
    "bumbar_hessian_model": (C.c_int, [vp, C.c_int, C.c_int64, C.c_int, C.c_int, vp, vp, C.c_int,
                                       vp, vp, vp, vp, vp, C.c_size_t, vp]),
    "bumbar_model_energies": (C.c_int, [vp, C.c_int, C.c_int64, C.c_int, C.c_int, vp, vp,
                                        C.c_int, vp]),
    "bumbar_sweep_static": (C.c_int, [vp, vp, C.c_int, C.c_int, C.c_int64, C.c_int64, vp, vp, vp,
                                      vp, vp, dp]),
    "bumbar_server_create": (C.c_int, [C.POINTER(ServerOptions), C.POINTER(C.c_void_p)]),
    "bumbar_server_submit": (C.c_int, [vp, C.POINTER(Request), u64p]),
    "bumbar_server_poll": (C.c_int, [vp, C.c_uint64, C.POINTER(C.c_int)]),
    "bumbar_server_wait": (C.c_int, [vp, C.c_uint64]),
    "bumbar_server_progress": (C.c_int, [vp, C.POINTER(C.c_int)]),
    "bumbar_server_result": (C.c_int, [vp, C.c_uint64, vp, C.POINTER(Stats), dp,
                                       C.POINTER(C.c_int)]),
    "bumbar_server_counters": (C.c_int, [vp, i64p, i64p, C.POINTER(C.c_size_t), i64p]),
    "bumbar_server_fused_counters": (C.c_int, [vp, i64p, i64p]),
    "bumbar_server_destroy": (None, [vp]),
}

_lib = None


def load():
    """Load libbumbar.so and declare its signatures (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
            "(the HIP library is required: there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
