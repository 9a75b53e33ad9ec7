"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances: FP64 single steps agree to 1e-12 (absolute, kT) or 1e-12
relative; full solves to 1e-9 kT (the FP64 target); bins, counts, widths and
bin maps are integers and must be identical.
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


def random_problem(K, N, seed, unsampled=()):
    g = np.random.default_rng(seed)
    Nk = np.zeros(K, dtype=np.int64)
    sampled = [k for k in range(K) if k not in unsampled]
    base = N // len(sampled)
    for k in sampled:
        Nk[k] = base
    Nk[sampled[0]] += N - Nk.sum()
    centres = g.uniform(-2, 2, K)
    kappa = g.uniform(0.5, 4, K)
    owner = np.repeat(np.arange(K), Nk)
    x = g.normal(centres[owner], 1 / np.sqrt(kappa[owner]))
    u = 0.5 * kappa[:, None] * (x[None, :] - centres[:, None]) ** 2
    return u, Nk, x


SHAPES = [(1, 37), (2, 129), (3, 1000), (8, 8000), (13, 515), (33, 130), (50, 4099), (56, 777),
          (57, 300), (64, 3001), (65, 2047),
          (100, 12345), (128, 4097), (200, 2500), (256, 1111), (300, 1500), (1000, 700)]


@pytest.mark.parametrize("K,N", SHAPES)
def test_single_sweep_matches_oracle(bm, K, N):
    say(f"sweep parity K={K} N={N}")
    u, Nk, _ = random_problem(K, N, seed=K * 7 + N)
    g = np.random.default_rng(1)
    f = np.concatenate([[0.0], g.normal(0, 0.3, K - 1)])
    fn_ref, lD_ref = oracle.sci_step(u, Nk, f, return_logD=True)
    fn, lD, S, st = bm.sweep(dev(u), Nk, f)
    fn, lD, S = fn.cpu().numpy(), lD.cpu().numpy(), S.cpu().numpy()
    assert np.max(np.abs(lD - lD_ref)) < 1e-12 * max(1.0, np.abs(lD_ref).max())
    assert np.max(np.abs(fn - fn_ref)) < 1e-12
    # S_i = N_i sum_n W_ni and the gradient norm
    W = oracle.weights(u, Nk, f)
    S_ref = Nk * W.sum(axis=0)
    samp = Nk > 0
    assert np.max(np.abs(S[samp] - S_ref[samp]) / S_ref[samp]) < 1e-12
    F_ref, g_ref = oracle.objective_gradient(u, Nk, f)
    assert abs(st["objective"] - F_ref) < 1e-10 * max(1.0, abs(F_ref))
    assert abs(st["grad_norm"] - np.linalg.norm(g_ref)) < 1e-9 * max(1.0, np.linalg.norm(g_ref))
    assert st["max_df"] == pytest.approx(np.max(np.abs(fn_ref - f)), rel=1e-9, abs=1e-13)


def test_sweep_with_padded_rows_and_unsampled_state(bm):
    import torch
    K, N = 6, 1001
    u, Nk, _ = random_problem(K, N, seed=3, unsampled=(2,))
    f = np.array([0.0, 0.4, 1.0, -0.3, 0.2, 0.1])
    fn_ref = oracle.sci_step(u, Nk, f)
    ld = 1040
    buf = torch.full((K, ld), float("nan"), dtype=torch.float64, device="cuda")
    buf[:, :N] = dev(u)
    fn, lD, S, st = bm.sweep(buf, Nk, f, ld=ld) if False else bm.sweep(buf[:, :N], Nk, f, ld=ld)
    assert np.max(np.abs(fn.cpu().numpy() - fn_ref)) < 1e-12


def test_robust_path_far_from_solution(bm):
    # a starting point 900 kT off makes some state sums underflow in double:
    # the fast path must flag it and the robust path give the oracle's step
    u, Nk, _ = random_problem(5, 2000, seed=4)
    f = np.array([0.0, 900.0, -5.0, 3.0, 0.0])
    fn_ref = oracle.sci_step(u, Nk, f)
    fn, lD, S, st = bm.sweep(dev(u), Nk, f)
    assert np.max(np.abs(fn.cpu().numpy() - fn_ref)) < 1e-9


@pytest.mark.parametrize("K,N", [(3, 500), (8, 4000), (64, 999), (100, 3000), (130, 777),
                                 (200, 1500), (256, 1001), (257, 600)])
def test_hessian_matches_oracle(bm, K, N):
    say(f"hessian parity K={K} N={N}")
    u, Nk, _ = random_problem(K, N, seed=K + N)
    f = np.concatenate([[0.0], np.random.default_rng(2).normal(0, 0.2, K - 1)])
    H_ref = oracle.hessian(u, Nk, f)
    ud = dev(u)
    fn, lD, S, _ = bm.sweep(ud, Nk, f)
    H = bm.hessian(ud, Nk, f, lD, S).cpu().numpy()
    scale = np.abs(H_ref).max()
    assert np.max(np.abs(H - H_ref)) < 1e-12 * scale


def test_weights_match_oracle(bm):
    u, Nk, _ = random_problem(7, 1234, seed=9, unsampled=(3,))
    f = np.array([0.0, 0.1, 0.5, 2.0, -0.2, 0.3, 0.0])
    W_ref = oracle.weights(u, Nk, f)
    ud = dev(u)
    _, lD, _, _ = bm.sweep(ud, Nk, f)
    W = bm.weights(ud, f, lD).cpu().numpy()
    assert np.max(np.abs(W - W_ref)) < 1e-13


@pytest.mark.parametrize("cfg", ["harmonic", "double_well", "unsampled"])
def test_plain_solve_matches_oracle(bm, cfg):
    say(f"plain solve parity {cfg}")
    if cfg == "harmonic":
        p = synth.harmonic_1d(K=8, Nk=1000, seed=0)
        u, Nk = p["u"], p["Nk"]
    elif cfg == "double_well":
        p = synth.double_well(K=40, Nk=500, seed=2)
        u, Nk = p["u"], p["Nk"]
    else:
        u, Nk, _ = random_problem(9, 3000, seed=5, unsampled=(0, 4))
    f_ref, info_ref = oracle.solve_mbar(u, Nk)
    f, info = bm.solve(dev(u), Nk, tol=1e-12)
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9
    assert info["grad_norm"] < 1e-6


@pytest.mark.parametrize("K,Nk,prec", [(140, 40, 0), (300, 30, 0), (300, 30, 1), (400, 20, 0),
                                        (700, 12, 1)])
def test_solve_large_reduced_system(bm, K, Nk, prec):
    # reduced Newton systems above the LDS solve's size use the blocked
    # Cholesky path (m = K - 1 > 136): m = 139, 299, 399, 699 give 3 to 11
    # blocks of 64, each with a ragged last block
    say(f"large-K solve K={K} Nk={Nk} precision={prec}")
    p = synth.harmonic_1d(K=K, Nk=Nk, seed=K)
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    f, info = bm.solve(dev(p["u"]), p["Nk"], tol=1e-12, precision=prec)
    say("finisher steps", info["finisher_steps"], "fallbacks", info["sci_fallbacks"],
        "hessians", info["hessians"])
    assert info["status"] == 0
    assert info["hessians"] >= 1
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9
    if prec == 0:
        # an FP64 Newton direction that is wrong shows up as SCI fallbacks
        assert info["sci_fallbacks"] == 0


@pytest.mark.parametrize("d", [1, 2])
def test_binning_bit_exact(bm, d):
    g = np.random.default_rng(30 + d)
    N = 20011
    xi = g.normal(0, 1, size=(N, d))
    xi[:300] = xi[300:600]  # duplicate points
    xi[600:700, 0] = xi[700, 0]  # ties along one axis
    q, lo, sc = oracle.quantize(xi)
    for n in [2, 100, 1000, 10000, 30000]:
        say(f"binning d={d} n={n}")
        m_ref, g_ref, _ = oracle.width_search(q, n)
        cells_ref, H_ref, sb_ref = oracle.histogram(q, m_ref)
        m, cells, H, sb = bm.bin_coordinates(xi, n)
        assert m == m_ref
        assert np.array_equal(cells.cpu().numpy().view(np.uint64), cells_ref)
        assert np.array_equal(H.cpu().numpy(), H_ref)
        assert np.array_equal(sb.cpu().numpy(), sb_ref)


@pytest.mark.parametrize("N", [1, 2, 7, 300, 4097, 8000, 16383, 16384, 16385, 65536, 65537])
def test_binning_small_1d(bm, N):
    # Up to 16384 samples the width search runs in one workgroup, and up to
    # 65536 keys the radix sort does (both one launch); 16385 and 65537 take
    # the multi-pass forms. Targets above N make g(1) < n (width 1).
    g = np.random.default_rng(1000 + N)
    xi = g.normal(0, 1, size=(N, 1))
    if N > 10:
        xi[: N // 10] = xi[N // 10: 2 * (N // 10)]  # duplicate points
    q, lo, sc = oracle.quantize(xi)
    for n in sorted({2, max(2, N // 3), max(2, N), N + 5}):
        say(f"binning small d=1 N={N} n={n}")
        m_ref, g_ref, _ = oracle.width_search(q, n)
        cells_ref, H_ref, sb_ref = oracle.histogram(q, m_ref)
        m, cells, H, sb = bm.bin_coordinates(xi, n)
        assert m == m_ref
        assert np.array_equal(cells.cpu().numpy().view(np.uint64), cells_ref)
        assert np.array_equal(H.cpu().numpy(), H_ref)
        assert np.array_equal(sb.cpu().numpy(), sb_ref)


@pytest.mark.parametrize("N", [5, 4096, 9000, 65536])
def test_binning_small_2d(bm, N):
    # 2-D cell keys sorted by the one-workgroup radix sort (64-bit keys)
    g = np.random.default_rng(2000 + N)
    xi = g.normal(0, 1, size=(N, 2))
    if N > 10:
        xi[: N // 10] = xi[N // 10: 2 * (N // 10)]
    q, lo, sc = oracle.quantize(xi)
    for n in sorted({2, max(2, N // 4), N + 1}):
        say(f"binning small d=2 N={N} n={n}")
        m_ref, g_ref, _ = oracle.width_search(q, n)
        cells_ref, H_ref, sb_ref = oracle.histogram(q, m_ref)
        m, cells, H, sb = bm.bin_coordinates(xi, n)
        assert m == m_ref
        assert np.array_equal(cells.cpu().numpy().view(np.uint64), cells_ref)
        assert np.array_equal(H.cpu().numpy(), H_ref)
        assert np.array_equal(sb.cpu().numpy(), sb_ref)


def test_binning_2d_heavy_tail(bm):
    # The 2-D probes visit the samples sorted by (q_y, q_x), a workgroup per
    # run of 2048: its cells lie in a band of grid rows, marked in LDS when
    # the band fits 8192 words, else in the global bitmap. A heavy-tailed y
    # makes the tail runs span many rows at fine widths (global marking)
    # while the bulk stays in LDS bands; every width must match the oracle.
    g = np.random.default_rng(77)
    N = 300007
    xi = np.stack([g.normal(0, 1, N), g.standard_cauchy(N)], axis=1)
    xi[:500] = xi[500:1000]  # duplicate points
    q, lo, sc = oracle.quantize(xi)
    for n in [100, 5000, 100000, 250000]:
        say(f"binning 2-D heavy tail n={n}")
        m_ref, g_ref, _ = oracle.width_search(q, n)
        cells_ref, H_ref, sb_ref = oracle.histogram(q, m_ref)
        m, cells, H, sb = bm.bin_coordinates(xi, n)
        assert m == m_ref
        assert np.array_equal(cells.cpu().numpy().view(np.uint64), cells_ref)
        assert np.array_equal(H.cpu().numpy(), H_ref)
        assert np.array_equal(sb.cpu().numpy(), sb_ref)


@pytest.mark.parametrize("N", [700001, 3000017, 12000007, 40000003])
def test_binning_large_1d(bm, N):
    # Large N evaluates fewer bisection levels per pass (4, 3, 2 and 2 here),
    # so the count kernel splits its chunks into 4, 8 and 16 streams. At
    # N = 7e5 the oracle's own search runs; above it (seconds per probe) the
    # GPU's m is checked by the bisection's end state g(m) >= n > g(m + 1)
    # with the oracle's g, and the histogram at m against the oracle's.
    g = np.random.default_rng(N)
    xi = g.normal(0, 1, size=(N, 1))
    xi[:1000] = xi[1000:2000]  # duplicate points
    q, lo, sc = oracle.quantize(xi)
    for n in ([100, 10000, 1000000] if N < 1000000 else [1000, 1000000]):
        say(f"binning d=1 N={N} n={n}")
        m, cells, H, _ = bm.bin_coordinates(xi, n)
        if N < 1000000:
            m_ref, _, _ = oracle.width_search(q, n)
            assert m == m_ref
        else:
            assert oracle.nonempty_bins(q, m) >= n > oracle.nonempty_bins(q, m + 1)
        cells_ref, H_ref, _ = oracle.histogram(q, m)
        assert np.array_equal(cells.cpu().numpy().view(np.uint64), cells_ref)
        assert np.array_equal(H.cpu().numpy(), H_ref)


def test_bumbar_solve_matches_oracle_1d(bm):
    p = synth.double_well(K=30, Nk=700, seed=5)
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    fo, info_o = oracle.bumbar(p["u"], p["Nk"], p["xi"], p["model_type"], p["coef"], tol=1e-11)
    f, info = bm.solve(dev(p["u"]), p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                       tol=1e-11)
    assert info["status"] == 0
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9
    say("schedule gpu", info["phase1_iters"], [c["refine"] for c in info["checks"]],
        "oracle", info_o["phase1"], [c["refine"] for c in info_o["checks"]])
    # replaying the oracle's schedule gives the oracle's binned trajectory
    flags = [c["refine"] for c in info_o["checks"]]
    f2, info2 = bm.solve(dev(p["u"]), p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                         tol=1e-11, replay=(info_o["phase1"], flags))
    gc = info2["checks"]
    oc = info_o["checks"]
    assert [c["P"] for c in gc] == [c["P"] for c in oc]
    assert [c["P_next"] for c in gc] == [c["P_next"] for c in oc]
    for a, b in zip(gc, oc):
        assert abs(a["s_n"] - b["s_n"]) <= 1e-9 * abs(b["s_n"]) + 1e-15
        assert abs(a["s_next"] - b["s_next"]) <= 1e-9 * abs(b["s_next"]) + 1e-15


@pytest.mark.parametrize("case", ["1d", "2d"])
def test_mean_representatives_replay_matches_oracle(bm, case):
    # plain u_kn (no model): the bin values of Eq. (1) are the bin means of u.
    # Replaying the oracle's schedule must give the oracle's binned trajectory
    # check by check: the same bins and the same Eq. (2) steps at n and n*inc.
    if case == "1d":
        p, n0 = synth.double_well(K=30, Nk=700, seed=6), 100
    else:
        p, n0 = synth.ladder_2d(K=16, Nk=1500, seed=3), 10
    say(f"MEAN replay {case} K={p['u'].shape[0]} N={p['u'].shape[1]}")
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    fo, info_o = oracle.bumbar(p["u"], p["Nk"], p["xi"], oracle.MODEL_NONE, None, tol=1e-11,
                               n0=n0)
    assert len(info_o["checks"]) >= 2
    flags = [c["refine"] for c in info_o["checks"]]
    f, info = bm.solve(dev(p["u"]), p["Nk"], xi=p["xi"], model=bm.MODEL_NONE, tol=1e-11, n0=n0,
                       replay=(info_o["phase1"], flags))
    assert info["status"] == 0
    assert info["phase1_iters"] == info_o["phase1"]
    gc, oc = info["checks"], info_o["checks"]
    assert len(gc) == len(oc)
    assert [c["P"] for c in gc] == [c["P"] for c in oc]
    assert [c["P_next"] for c in gc] == [c["P_next"] for c in oc]
    # Eq. (2) is a difference quotient of iterates: the bin means are summed
    # in another order on each side (about 1e-16 relative), which leaves the
    # iterates about 1e-14 kT apart after hundreds of steps, so a step s of
    # 1e-5 agrees to about 1e-14 absolute, not to 1e-9 relative
    for a, b in zip(gc, oc):
        assert abs(a["s_n"] - b["s_n"]) <= 1e-9 * abs(b["s_n"]) + 1e-12
        assert abs(a["s_next"] - b["s_next"]) <= 1e-9 * abs(b["s_next"]) + 1e-12
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9


def test_bumbar_solve_mean_representatives_2d(bm):
    p = synth.ladder_2d(K=12, Nk=300, seed=1)
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    f, info = bm.solve(dev(p["u"]), p["Nk"], xi=p["xi"], model=bm.MODEL_NONE, tol=1e-11)
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9
    f2, info2 = bm.solve(dev(p["u"]), p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                         tol=1e-11)
    assert np.max(np.abs(f2.cpu().numpy() - f_ref)) < 1e-9


def test_representative_choices(bm):
    # AUTO with a model is CENTRE (bitwise); MEAN with a model given uses the
    # bin means; all reach the unbinned solution
    p = synth.harmonic_1d(K=10, Nk=400, seed=12)
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    kw = dict(xi=p["xi"], model=p["model_type"], coef=p["coef"], tol=1e-11)
    fa, _ = bm.solve(dev(p["u"]), p["Nk"], represent=bm.REPRESENT_AUTO, **kw)
    fc, _ = bm.solve(dev(p["u"]), p["Nk"], represent=bm.REPRESENT_CENTRE, **kw)
    fm, _ = bm.solve(dev(p["u"]), p["Nk"], represent=bm.REPRESENT_MEAN, **kw)
    assert np.array_equal(fa.cpu().numpy(), fc.cpu().numpy())
    # MEAN with the model given is MEAN without it (the model is not used)
    fm0, _ = bm.solve(dev(p["u"]), p["Nk"], xi=p["xi"], tol=1e-11)
    assert np.array_equal(fm.cpu().numpy(), fm0.cpu().numpy())
    for f in (fc, fm):
        assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9
    with pytest.raises(bm.BumbarError):
        bm.solve(dev(p["u"]), p["Nk"], xi=p["xi"], represent=bm.REPRESENT_CENTRE, tol=1e-11)


def test_reweight_matches_oracle(bm):
    p = synth.harmonic_1d(K=4, Nk=300, seed=6)
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    lD_ref = oracle.log_denominator(p["u"], p["Nk"], f_ref)
    f, info = bm.solve(dev(p["u"]), p["Nk"], tol=1e-12, want_logD=True)
    ut = 0.5 * 2.0 * (p["xi"][:, 0] - 0.3) ** 2
    pr = bm.reweight(dev(ut), info["logD"]).cpu().numpy()
    assert np.max(np.abs(pr - oracle.reweight(ut, lD_ref))) < 1e-12 * max(1, pr.max())


def test_deterministic_repeat(bm):
    u, Nk, _ = random_problem(100, 50000, seed=11)
    f = np.zeros(100)
    a = bm.sweep(dev(u), Nk, f)[0].cpu().numpy()
    b = bm.sweep(dev(u), Nk, f)[0].cpu().numpy()
    assert np.array_equal(a, b)


def test_invalid_inputs_raise(bm):
    u, Nk, _ = random_problem(4, 100, seed=1)
    with pytest.raises(bm.BumbarError):
        bm.solve(dev(u), Nk + 1)  # sum N_k != N
    bad = u.copy()
    bad[1, 5] = np.nan
    with pytest.raises(bm.BumbarError):
        bm.solve(dev(bad), Nk)


@pytest.mark.parametrize("K,N,pad", [(5, 999, 0), (100, 3001, 0), (300, 2000, 0), (64, 1024, 0),
                                     (256, 4097, 0), (100, 1000, 1), (13, 777, 3)])
def test_fp32_input_sweep_matches_oracle_on_widened_values(bm, K, N, pad):
    # FP32 u is widened to FP64 on load (the register-tiled sweep for K <= 256,
    # with 8-byte loads when rows are aligned, element loads otherwise): the
    # exact reference is the oracle on the float-rounded values. pad > 0 gives
    # a row stride N + pad (unaligned rows).
    import torch
    u, Nk, _ = random_problem(K, N, seed=K + 3 * N)
    u32 = u.astype(np.float32)
    f = np.concatenate([[0.0], np.random.default_rng(3).normal(0, 0.2, K - 1)])
    fn_ref, lD_ref = oracle.sci_step(u32.astype(np.float64), Nk, f, return_logD=True)
    ut = torch.zeros((K, N + pad), dtype=torch.float32, device="cuda")
    ut[:, :N] = torch.as_tensor(u32).cuda()
    fn, lD, S, st = bm.sweep(ut[:, :N], Nk, f)
    assert np.max(np.abs(fn.cpu().numpy() - fn_ref)) < 1e-12
    assert np.max(np.abs(lD.cpu().numpy() - lD_ref)) < 1e-12 * max(1.0, np.abs(lD_ref).max())
    F_ref, g_ref = oracle.objective_gradient(u32.astype(np.float64), Nk, f)
    assert abs(st["objective"] - F_ref) < 1e-10 * max(1.0, abs(F_ref))


@pytest.mark.parametrize("K,Nk,xi", [(8, 1500, False), (120, 60, True), (256, 20, False)])
def test_fp32_storage_solve_mixed(bm, K, Nk, xi):
    # mixed precision on FP32 storage with K <= 256: Newton on FP32-exponential
    # sweeps of the stored u (no copy), then FP64 refinement: the oracle's
    # solution of the rounded problem to 1e-9 kT
    p = synth.harmonic_1d(K=K, Nk=Nk, seed=K + 7)
    u32 = p["u"].astype(np.float32)
    f_ref, _ = oracle.solve_mbar(u32.astype(np.float64), p["Nk"])
    kw = dict(xi=p["xi"], model=p["model_type"], coef=p["coef"]) if xi else {}
    plan = bm.plan(K, p["N"], u_dtype=bm.F32, precision=bm.PREC_MIXED)
    assert plan["stage32"] == 4  # BUMBAR_STAGE32_STORED
    f, info = bm.solve(dev(u32), p["Nk"], tol=1e-11, precision=bm.PREC_MIXED, **kw)
    say(f"fp32 storage mixed K={K}: mixed steps {info['mixed_steps']}, "
        f"all {info['finisher_steps']}")
    assert info["status"] == 0 and info["mixed_steps"] >= 1
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9


@pytest.mark.parametrize("K,Nk", [(8, 1500), (120, 60), (256, 20)])
def test_fp32_storage_solve_fp64(bm, K, Nk):
    # FP64 solve of an FP32-stored matrix (register-tiled sweeps for K <= 256):
    # the oracle's solution of the rounded problem to 1e-9 kT
    p = synth.harmonic_1d(K=K, Nk=Nk, seed=K)
    u32 = p["u"].astype(np.float32)
    f_ref, _ = oracle.solve_mbar(u32.astype(np.float64), p["Nk"])
    plan = bm.plan(K, p["N"], u_dtype=bm.F32)
    assert plan["sweep"] == 0  # BUMBAR_SWEEP_REGISTER
    f, info = bm.solve(dev(u32), p["Nk"], tol=1e-11)
    assert info["status"] == 0
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9


@pytest.mark.parametrize("cfg", ["harmonic", "double_well", "ladder"])
def test_mixed_precision_solve_matches_fp64_oracle(bm, cfg):
    say(f"mixed precision solve {cfg}")
    if cfg == "harmonic":
        p = synth.harmonic_1d(K=8, Nk=1500, seed=2)
    elif cfg == "double_well":
        p = synth.double_well(K=50, Nk=400, seed=7)
    else:
        p = synth.ladder_2d(K=120, Nk=60, seed=3)
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    f, info = bm.solve(dev(p["u"]), p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                       precision=bm.PREC_MIXED, tol=1e-11)
    err = np.max(np.abs(f.cpu().numpy() - f_ref))
    say(f"  mixed steps {info['mixed_steps']} fp64 steps {info['finisher_steps'] - info['mixed_steps']}"
        f" err {err:.2e}")
    assert info["mixed_steps"] >= 1
    assert err < 1e-9


def test_mixed_precision_fp32_stage_accuracy(bm):
    # stopping right after the FP32 stage (loose tol) already lands within
    # 1e-4 kT; the refinement is what reaches the FP64 tolerance
    p = synth.double_well(K=40, Nk=500, seed=8)
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    f, info = bm.solve(dev(p["u"]), p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                       precision=bm.PREC_MIXED, tol=1e-3, mixed_tol=1e-3)
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-3


def test_hessian_fp32_input(bm):
    import torch
    K, N = 70, 2000
    u, Nk, _ = random_problem(K, N, seed=21)
    u32 = u.astype(np.float32)
    f = np.concatenate([[0.0], np.random.default_rng(5).normal(0, 0.2, K - 1)])
    H_ref = oracle.hessian(u32.astype(np.float64), Nk, f)
    ud = torch.as_tensor(u32).cuda()
    fn, lD, S, _ = bm.sweep(ud, Nk, f)
    H = bm.hessian(ud, Nk, f, lD, S).cpu().numpy()
    assert np.max(np.abs(H - H_ref)) < 1e-12 * np.abs(H_ref).max()


def test_trace_file_records_the_schedule(bm, tmp_path):
    # trace_path: one line per phase-2 check (the same values as the checks
    # in the statistics) and a summary line; appended on every solve
    p = synth.double_well(K=20, Nk=2000, seed=5)
    path = str(tmp_path / "trace.txt")
    u = dev(p["u"])
    kw = dict(xi=p["xi"], model=p["model_type"], coef=p["coef"], tol=1e-10)
    f, info = bm.solve(u, p["Nk"], trace_path=path, **kw)
    assert info["status"] == 0 and info["n_checks"] >= 1
    lines = open(path).read().splitlines()
    checks = [l.split() for l in lines if l.startswith("check ")]
    assert len(checks) == info["n_checks"] == len(info["checks"])
    for row, c in zip(checks, info["checks"]):
        assert (int(row[2]), int(row[3]), int(row[4])) == (c["n"], c["P"], c["P_next"])
        assert float(row[5]) == c["s_n"] and float(row[6]) == c["s_next"]
        assert (int(row[7]), int(row[8])) == (c["refine"], c["stop"])
    summ = [l for l in lines if l.startswith("summary ")]
    assert len(summ) == 1 and f"phase1_iters={info['phase1_iters']}" in summ[0]
    # a second solve appends; a solve without a trace leaves the file alone
    bm.solve(u, p["Nk"], trace_path=path, checks_capacity=1, **kw)
    bm.solve(u, p["Nk"], **kw)
    assert sum(1 for l in open(path) if l.startswith("summary ")) == 2
