"""bumbar_sweep_static (no device allocation) against bumbar_sweep, through the C ABI.

Two calls in a row, the second on a smaller problem, so stale contents of the
shared fixed scratch array from the first call must not leak into the second.
Both entry points run the same kernels with the same launch shapes, so the
results must agree to the bit.
"""
import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_03541_amd as bm
    from paper_2609_03541_amd import _capi
    ctx = bm.Context()
    return torch, bm, _capi.load(), ctx


def problem(torch, K, N, seed, dtype):
    g = np.random.default_rng(seed)
    Nk = np.full(K, N // K, dtype=np.int64)
    Nk[0] += N - Nk.sum()
    if K > 2:
        Nk[1] += Nk[2]
        Nk[2] = 0  # one unsampled state
    x0 = g.uniform(-2, 2, K)
    kap = g.uniform(0.5, 4, K)
    x = g.normal(0, 1.5, N)
    u = 0.5 * kap[:, None] * (x[None, :] - x0[:, None]) ** 2
    f = np.concatenate([[0.0], g.normal(0, 0.3, K - 1)])
    dev = torch.device("cuda")
    return (torch.tensor(u, dtype=dtype, device=dev), torch.tensor(Nk, device=dev),
            torch.tensor(f, device=dev))


def run_pair(torch, bm, lib, ctx, u, Nk, f, with_stats):
    K, N = u.shape
    code = bm.F64 if u.dtype == torch.float64 else bm.F32
    p = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    nb = C.c_size_t()
    assert lib.bumbar_query_workspace(ctx.h, K, N, 0, None, C.byref(nb)) == 0
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    outs = []
    for static in (False, True):
        fn = torch.empty(K, dtype=torch.float64, device="cuda")
        lD = torch.empty(N, dtype=torch.float64, device="cuda")
        S = torch.empty(K, dtype=torch.float64, device="cuda")
        st = (C.c_double * 4)() if with_stats else None
        stp = C.cast(st, C.POINTER(C.c_double)) if with_stats else None
        if static:
            rc = lib.bumbar_sweep_static(ctx.h, p(u), code, K, N, N, p(Nk), p(f), p(fn), p(lD),
                                         p(S), stp)
        else:
            rc = lib.bumbar_sweep(ctx.h, p(u), code, K, N, N, p(Nk), p(f), p(ws), nb.value,
                                  p(fn), p(lD), p(S), stp)
        assert rc == 0, ctx.error()
        torch.cuda.synchronize()
        outs.append((fn.cpu().numpy(), lD.cpu().numpy(), S.cpu().numpy(),
                     list(st) if with_stats else None))
    return outs


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("with_stats", [True, False])
def test_static_sweep_equals_workspace_sweep(env, dtype_name, with_stats):
    torch, bm, lib, ctx = env
    dtype = torch.float64 if dtype_name == "f64" else torch.float32
    # second call smaller in K and N than the first
    for K, N, seed in [(200, 300007, 1), (37, 4099, 2)]:
        say(f"static sweep {dtype_name} stats={with_stats} K={K} N={N}")
        u, Nk, f = problem(torch, K, N, seed, dtype)
        (a_f, a_l, a_s, a_st), (b_f, b_l, b_s, b_st) = run_pair(torch, bm, lib, ctx, u, Nk, f,
                                                                with_stats)
        assert np.array_equal(a_f, b_f)
        assert np.array_equal(a_l, b_l)
        samp = Nk.cpu().numpy() > 0
        assert np.array_equal(a_s[samp], b_s[samp])
        if with_stats:
            assert a_st == b_st


def test_static_sweep_rejects_sizes_beyond_its_limits(env):
    torch, bm, lib, ctx = env
    u, Nk, f = problem(torch, 8, 1000, 3, torch.float64)
    out = torch.empty(300, dtype=torch.float64, device="cuda")
    lD = torch.empty(1000, dtype=torch.float64, device="cuda")
    p = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    # K above the limit (the pointers are never dereferenced: the call fails first)
    rc = lib.bumbar_sweep_static(ctx.h, p(u), bm.F64, 300, 1000, 1000, p(Nk), p(f), p(out),
                                 p(lD), None, None)
    assert rc == bm.EINVAL and "K <=" in ctx.error()
    rc = lib.bumbar_sweep_static(ctx.h, p(u), bm.F64, 8, (1 << 22) + 1, (1 << 22) + 1, p(Nk),
                                 p(f), p(out), p(lD), None, None)
    assert rc == bm.EINVAL
    rc = lib.bumbar_sweep_static(ctx.h, p(u), bm.F64, 8, 1000, 1000, p(Nk), p(f), p(out), None,
                                 None, None)
    assert rc == bm.EINVAL
