"""Input element types at the boundary: FP32 coordinates.

bumbar_solve takes xi as FP64 or FP32; FP32 coordinates are widened exactly
to FP64 inside the library, so a solve given FP32 xi is bitwise the solve
given the same values as FP64, on every path that reads xi (binning in 1-D
and 2-D, model energies in the kernels, the product-grid passes), and it
reaches the oracle's solution of that problem.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build()
    import paper_2609_03541_amd as bm
    return bm


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def model_u(bm, xi64, p):
    return bm.model_energies(xi64, p["coef"], p["model_type"], p["K"])


@pytest.mark.parametrize("prec", [0, 1])
def test_fp32_xi_on_the_fly_2d(bm, prec):
    # Mueller-Brown windows on a 12 x 12 grid: model energies from (x, y),
    # 2-D binning, and the factored product-grid passes all read xi
    p = synth.muller_brown_grid(G=12, Nk=120, seed=4)
    x32 = p["xi"].astype(np.float32)
    x64 = x32.astype(np.float64)
    kw = dict(model=p["model_type"], coef=p["coef"], tol=1e-11, precision=prec)
    fa, ia = bm.solve(None, p["Nk"], xi=dev(x32), **kw)
    fb, ib = bm.solve(None, p["Nk"], xi=dev(x64), **kw)
    say("fp32 xi 2-D precision", prec, "grid sweeps", ia["grid_sweeps"])
    assert ia["status"] == 0 and ib["status"] == 0
    assert np.array_equal(fa.cpu().numpy(), fb.cpu().numpy())
    u = model_u(bm, x64, p).cpu().numpy()
    f_ref, _ = oracle.solve_mbar(u, p["Nk"])
    assert np.max(np.abs(fa.cpu().numpy() - f_ref)) < (1e-9 if prec == 0 else 1e-6)


def test_fp32_xi_stored_u_1d_binning(bm):
    # stored u with 1-D binning coordinates in FP32 (bin-centre representatives)
    p = synth.double_well(K=40, Nk=500, seed=6)
    x32 = p["xi"].astype(np.float32)
    x64 = x32.astype(np.float64)
    u = model_u(bm, x64, p)
    kw = dict(model=p["model_type"], coef=p["coef"], tol=1e-11)
    fa, ia = bm.solve(u, p["Nk"], xi=x32, **kw)
    fb, ib = bm.solve(u, p["Nk"], xi=x64, **kw)
    assert ia["status"] == 0 and ia["n_checks"] >= 1
    assert np.array_equal(fa.cpu().numpy(), fb.cpu().numpy())
    f_ref, _ = oracle.solve_mbar(u.cpu().numpy(), p["Nk"])
    assert np.max(np.abs(fa.cpu().numpy() - f_ref)) < 1e-9


def test_fp32_xi_needs_its_workspace(bm):
    # a workspace sized for FP64 coordinates is refused for FP32 ones
    import ctypes as C
    import torch
    p = synth.double_well(K=8, Nk=200, seed=7)
    ctx = bm.context()
    opts = bm.default_options(binning=1, represent=bm.REPRESENT_CENTRE)
    nb = ctx.query_workspace(p["K"], p["N"], 1, opts)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")  # exactly the FP64 size
    x32 = dev(p["xi"].astype(np.float32))
    u = dev(p["u"])
    nk = dev(p["Nk"])
    coef = dev(p["coef"])
    f = torch.empty(p["K"], dtype=torch.float64, device="cuda")
    rc = ctx.lib.bumbar_solve(ctx.h, C.c_void_p(u.data_ptr()), bm.F64, p["K"], p["N"],
                              C.c_void_p(nk.data_ptr()), C.c_void_p(x32.data_ptr()), bm.F32, 1,
                              int(p["model_type"]), C.c_void_p(coef.data_ptr()), None,
                              C.byref(opts), C.c_void_p(ws.data_ptr()), ws.numel(),
                              C.c_void_p(f.data_ptr()), None, None, None)
    assert rc == bm.ENOMEM
    torch.cuda.synchronize()
