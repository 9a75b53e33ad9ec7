"""GPU parity at the benchmark's full size and at large N, where every
workgroup of the persistent sweep walks many column tiles.

The double-well umbrella workload (K = 100 windows, N = 1e6 samples, u_kn
100 x 1e6 FP64) is small enough for the FP64 oracle to take whole sweeps, so
single sweeps are compared element by element (1e-12, as the small-size
parity tests). A full solve is checked against the oracle's own certified
solution started from the GPU result (1e-9 kT), and by the oracle's
fixed-point residual at the GPU result.
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


def harmonic(K, N, seed, unsampled=()):
    g = np.random.default_rng(seed)
    Nk = np.zeros(K, dtype=np.int64)
    sampled = [k for k in range(K) if k not in unsampled]
    Nk[sampled] = N // len(sampled)
    Nk[sampled[0]] += N - Nk.sum()
    centres = np.linspace(-2, 2, K)
    kappa = g.uniform(4, 40, K)
    owner = np.repeat(np.arange(K), Nk)
    x = g.normal(centres[owner], 1 / np.sqrt(kappa[owner]))
    u = 0.5 * kappa[:, None] * (x[None, :] - centres[:, None]) ** 2
    return u, Nk


def check_sweep(bm, u, Nk, f, want_logD):
    fn_ref, lD_ref = oracle.sci_step(u, Nk, f, return_logD=True)
    fn, lD, S, st = bm.sweep(dev(u), Nk, f, want_logD=want_logD)
    fn, S = fn.cpu().numpy(), S.cpu().numpy()
    assert np.max(np.abs(fn - fn_ref)) < 1e-12
    if want_logD:
        lD = lD.cpu().numpy()
        assert np.max(np.abs(lD - lD_ref)) < 1e-12 * max(1.0, np.abs(lD_ref).max())
    F_ref, g_ref = oracle.objective_gradient(u, Nk, f)
    assert abs(st["objective"] - F_ref) < 1e-10 * max(1.0, abs(F_ref))
    assert abs(st["grad_norm"] - np.linalg.norm(g_ref)) < 1e-9 * max(1.0, np.linalg.norm(g_ref))
    # S_i = N_i sum_n W_ni
    samp = Nk > 0
    S_ref = Nk * oracle.weights(u, Nk, f).sum(axis=0)
    assert np.max(np.abs(S[samp] - S_ref[samp]) / S_ref[samp]) < 1e-12


# K across the sweep's row shapes (32 < K <= 128); even N keeps u 16-byte
# aligned (vector loads), odd N takes the scalar-load path; N leaves a ragged
# last tile; some states unsampled
LARGE = [(33, 70002, ()), (64, 65728, ()), (65, 90018, (0, 31)), (77, 140004, (5,)),
        (100, 300008, ()), (100, 131086, (99,)), (128, 200006, ()), (113, 98306, (1, 2)),
        (100, 300007, ()), (77, 140003, (5,))]


@pytest.mark.parametrize("K,N,unsampled", LARGE)
@pytest.mark.parametrize("want_logD", [True, False])
def test_large_sweep_matches_oracle(bm, K, N, unsampled, want_logD):
    say(f"large sweep K={K} N={N} unsampled={unsampled} logD={want_logD}")
    u, Nk = harmonic(K, N, seed=K + N, unsampled=unsampled)
    g = np.random.default_rng(2)
    f = np.concatenate([[0.0], g.normal(0, 0.3, K - 1)])
    check_sweep(bm, u, Nk, f, want_logD)


@pytest.fixture(scope="module")
def double_well():
    say("generating the double-well workload K=100 N=1e6")
    return synth.double_well(K=100, Nk=10000, seed=1)


def test_full_size_double_well_sweep(bm, double_well):
    p = double_well
    say("full-size sweep K=100 N=1e6")
    g = np.random.default_rng(5)
    f = np.concatenate([[0.0], np.cumsum(g.normal(0, 0.5, 99))])
    check_sweep(bm, p["u"], p["Nk"], f, want_logD=True)


def test_full_size_double_well_solve(bm, double_well):
    import torch
    p = double_well
    say("full-size solve K=100 N=1e6 (adaptive binning + Newton)")
    u = dev(p["u"])
    f, info = bm.solve(u, p["Nk"], xi=dev(p["xi"]), model=bm.MODEL_HARMONIC,
                       coef=dev(p["coef"]), tol=1e-10)
    assert info["status"] == 0
    fh = f.cpu().numpy()
    del u
    torch.cuda.empty_cache()
    res = np.max(np.abs(oracle.sci_step(p["u"], p["Nk"], fh) - fh))
    say(f"  oracle fixed-point residual at the GPU result: {res:.3e}")
    assert res < 1e-9
    f_ref, inf = oracle.solve_mbar(p["u"], p["Nk"], f_init=fh, newton_tol=1e-12)
    assert inf["rc"] == 0
    assert np.max(np.abs(fh - f_ref)) < 1e-9
