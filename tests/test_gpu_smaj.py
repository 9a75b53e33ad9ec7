"""GPU parity of the sample-major path (256 < K <= 1024) against the FP64 oracle.

The single sweep over the sample-major copy (FP64, or FP32 storage widened)
agrees with the oracle's step to 1e-12 (it differs only in summation order
and a 64-entry-table exponential, relative error ~3e-16); solves through it
(FP64, and mixed precision with its FP32-arithmetic stage followed by FP64
refinement) reach the oracle's fixed point to 1e-9 kT. FP32 storage makes
the FP32-rounded energies the problem: the oracle is run on them, widened.
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


def problem(K, N, seed, unsampled=()):
    g = np.random.default_rng(seed)
    Nk = np.zeros(K, dtype=np.int64)
    sampled = [k for k in range(K) if k not in unsampled]
    for k in sampled:
        Nk[k] = N // len(sampled)
    Nk[sampled[0]] += N - Nk.sum()
    x0 = g.uniform(-2, 2, K)
    kap = g.uniform(0.5, 4, K)
    owner = np.repeat(np.arange(K), Nk)
    x = g.normal(x0[owner], 1 / np.sqrt(kap[owner]))
    u = 0.5 * kap[:, None] * (x[None, :] - x0[:, None]) ** 2
    f = np.concatenate([[0.0], g.normal(0, 0.3, K - 1)])
    return u, Nk, f


def row_len(K):
    # rows of 64 J, J the smallest of 5, 6, 8, 10, 12, 14, 16 with K <= 64 J
    return 64 * next(j for j in (5, 6, 8, 10, 12, 14, 16) if K <= 64 * j)


SHAPES = [(257, 1001, ()), (300, 4099, (5,)), (511, 777, ()), (640, 1500, (0, 3)),
          (1000, 2003, ()), (1024, 333, (1023,))]


@pytest.mark.parametrize("K,N,unsampled", SHAPES)
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_sample_major_sweep_matches_oracle(bm, K, N, unsampled, storage):
    import torch
    say(f"sample-major sweep {storage} K={K} N={N} unsampled={unsampled}")
    u, Nk, f = problem(K, N, seed=K + N, unsampled=unsampled)
    if storage == "f32":
        u = u.astype(np.float32).astype(np.float64)  # the problem is the FP32 storage
    fn_ref, lD_ref = oracle.sci_step(u, Nk, f, return_logD=True)
    ut = dev(u) if storage == "f64" else dev(u.astype(np.float32))
    copy = bm.sample_major(ut)
    assert copy.data.numel() == N * row_len(K)
    fn, lD, S, st = bm.sweep(copy, Nk, f)
    torch.cuda.synchronize()
    fn, lD, S = fn.cpu().numpy(), lD.cpu().numpy(), S.cpu().numpy()
    assert np.max(np.abs(lD - lD_ref)) < 1e-12 * max(1.0, np.abs(lD_ref).max())
    assert np.max(np.abs(fn - fn_ref)) < 1e-12
    W = oracle.weights(u, Nk, f)
    S_ref = Nk * W.sum(axis=0)
    samp = Nk > 0
    assert np.max(np.abs(S[samp] - S_ref[samp]) / S_ref[samp]) < 1e-12
    F_ref, g_ref = oracle.objective_gradient(u, Nk, f)
    assert abs(st["objective"] - F_ref) < 1e-10 * max(1.0, abs(F_ref))
    assert abs(st["grad_norm"] - np.linalg.norm(g_ref)) < 1e-9 * max(1.0, np.linalg.norm(g_ref))


def test_sample_major_copy_layout(bm):
    # the copy is u transposed, rows padded to 64 J (J = 5 for K = 300) with +inf
    import torch
    K, N = 300, 131
    u = np.random.default_rng(7).normal(size=(K, N))
    c = bm.sample_major(dev(u)).data.cpu().numpy().reshape(N, 320)
    assert np.array_equal(c[:, :K], u.T)
    assert np.all(np.isinf(c[:, K:])) and np.all(c[:, K:] > 0)
    torch.cuda.synchronize()


def test_sample_major_robust_path(bm):
    # a start 900 kT off underflows state sums: the sweep is redone on the
    # robust two-pass path reading the copy with its strides
    u, Nk, f = problem(300, 2000, seed=11)
    f = f.copy()
    f[7] = 900.0
    fn_ref = oracle.sci_step(u, Nk, f)
    fn, lD, S, st = bm.sweep(bm.sample_major(dev(u)), Nk, f)
    assert np.max(np.abs(fn.cpu().numpy() - fn_ref)) < 1e-9


@pytest.mark.parametrize("K,Nk,storage,prec", [(300, 30, "f64", 0), (400, 20, "f32", 0),
                                                (400, 20, "f32", 1), (700, 12, "f64", 1),
                                                (1000, 8, "f32", 1)])
def test_solve_through_sample_major(bm, K, Nk, storage, prec):
    say(f"sample-major solve K={K} Nk={Nk} {storage} precision={prec}")
    p = synth.harmonic_1d(K=K, Nk=Nk, seed=K + 1)
    u = p["u"] if storage == "f64" else p["u"].astype(np.float32)
    plan = bm.plan(K, K * Nk, u_dtype=bm.F64 if storage == "f64" else bm.F32, precision=prec)
    assert plan["copy_bytes"] > 0
    f_ref, _ = oracle.solve_mbar(u.astype(np.float64), p["Nk"])
    f, info = bm.solve(dev(u), p["Nk"], tol=1e-12, precision=prec)
    say("finisher", info["finisher_steps"], "mixed", info["mixed_steps"], "fallbacks",
        info["sci_fallbacks"], "hessians", info["hessians"])
    assert info["status"] == 0
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9
    if prec == 1:
        assert info["mixed_steps"] >= 1


def test_solve_copy_off_equals_copy_on(bm):
    p = synth.harmonic_1d(K=320, Nk=25, seed=5)
    fa, _ = bm.solve(dev(p["u"]), p["Nk"], tol=1e-12)
    fb, _ = bm.solve(dev(p["u"]), p["Nk"], tol=1e-12, sample_major=0)
    assert np.max(np.abs(fa.cpu().numpy() - fb.cpu().numpy())) < 1e-10


def test_newton_from_poor_start_weak_overlap(bm):
    # A weak-overlap ladder with K > 256 (sample-major sweeps, FP16-core
    # Newton Hessian) from a poor start (one SCI step from f = 0): Newton
    # needs damped steps there, and the finisher may stop only on a full
    # step, so the result must still be the oracle's fixed point.
    p = synth.ladder_2d(K=300, Nk=40, seed=9, delta=1.2)  # neighbour overlap 2 Phi(-0.6) = 0.55
    f_ref, info_ref = oracle.solve_mbar(p["u"], p["Nk"])
    f, info = bm.solve(dev(p["u"]), p["Nk"], tol=1e-11, sci_switch=1e9)
    say("damped", info["damped_steps"], "fallbacks", info["sci_fallbacks"], "newton",
        info["finisher_steps"], "oracle residual", info_ref["residual"])
    assert info["status"] == 0
    assert info["damped_steps"] + info["sci_fallbacks"] >= 1
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9


def test_nan_in_u_is_refused(bm):
    # the solve's copy is checked for NaN once; a caller's copy in every sweep
    p = synth.harmonic_1d(K=300, Nk=10, seed=3)
    u = p["u"].copy()
    u[123, 456] = np.nan
    with pytest.raises(bm.BumbarError) as e:
        bm.solve(dev(u), p["Nk"], tol=1e-10)
    assert e.value.code == bm.EINVAL
    with pytest.raises(bm.BumbarError):
        bm.sweep(bm.sample_major(dev(u)), p["Nk"], np.zeros(300))
