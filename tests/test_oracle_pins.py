"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

The paper prints no worked example, so each oracle function is tied to a
closed form, an invariant, a special case or an independent high-precision
computation (see tests/brute.py). Each pin is chosen so that a plausible
mistake (a dropped ln N_k, a wrong sign, a transposed operand, a missing
gauge) fails at least one of them.
"""
import math

import numpy as np
import pytest

import synth
from tests import brute


def constructed_exact(seed, K=4, L=6):
    """Exact MBAR problem: f_k - f_0 = a_k - a_0 by construction.

    Finite support {x_1..x_L}; state k holds c_kx > 0 copies of x and
    u_k(x) = -ln(c_kx / N_k) + a_k. Then sum_k N_k exp(f_k - u_k(x)) with
    f_k = a_k is sum_k c_kx = C_x, and the MBAR equation for state i reduces
    to sum_x (c_ix / N_i) = 1.
    """
    g = np.random.Generator(np.random.PCG64(seed))
    c = g.integers(1, 6, size=(K, L))
    a = g.normal(0.0, 3.0, K)
    Nk = c.sum(axis=1)
    cols = []
    for k in range(K):
        for x in range(L):
            cols += [x] * int(c[k, x])
    xs = np.array(cols)
    u = np.empty((K, len(xs)))
    for k in range(K):
        u[k] = -np.log(c[k, xs] / Nk[k]) + a[k]
    return u, Nk, a - a[0]


@pytest.mark.parametrize("seed", range(5))
def test_p1_constructed_exact(orc, seed):
    u, Nk, f_true = constructed_exact(seed, K=3 + seed, L=5 + seed)
    f, info = orc.solve_mbar(u, Nk)
    assert info["rc"] == 0
    assert np.max(np.abs(f - f_true)) < 1e-12


def test_p1_constructed_exact_sci_fixed_point(orc):
    # one SCI step from the exact answer returns the exact answer
    u, Nk, f_true = constructed_exact(11, K=5, L=7)
    f1 = orc.sci_step(u, Nk, f_true)
    assert np.max(np.abs(f1 - f_true)) < 1e-13


@pytest.mark.parametrize("seed", range(3))
def test_p2_two_states_reduce_to_bar(orc, seed):
    p = synth.harmonic_1d(K=2, Nk=[300 + 50 * seed, 200], seed=10 + seed)
    u, Nk = p["u"], p["Nk"]
    f, info = orc.solve_mbar(u, Nk)
    df = brute.bar_bisection(u[0], u[1], int(Nk[0]), int(Nk[1]))
    assert abs(f[1] - df) < 1e-11


def test_p3_harmonic_analytic(orc):
    """f_k - f_0 = 1/2 ln(kappa_k / kappa_0) for harmonic wells at beta = 1 (statistical)."""
    devs = []
    for seed in range(8):
        p = synth.harmonic_1d(K=8, Nk=4000, seed=seed)
        f, _ = orc.solve_mbar(p["u"], p["Nk"])
        devs.append(f - 0.5 * np.log(p["kappa"] / p["kappa"][0]))
    devs = np.array(devs)[:, 1:]
    mean = devs.mean(axis=0)
    sem = devs.std(axis=0, ddof=1) / math.sqrt(devs.shape[0])
    assert np.all(np.abs(mean) < 4 * sem + 1e-3)
    assert np.max(np.abs(devs)) < 0.1


def test_p3_harmonic_large_sample(orc):
    p = synth.harmonic_1d(K=8, Nk=100000, seed=0)
    f, _ = orc.solve_mbar(p["u"], p["Nk"])
    assert np.max(np.abs(f - 0.5 * np.log(p["kappa"] / p["kappa"][0]))) < 0.02


def test_p4_invariants(orc):
    p = synth.harmonic_1d(K=6, Nk=[50, 80, 0, 60, 70, 40], seed=3)
    u, Nk = p["u"], p["Nk"]
    rng = np.random.default_rng(0)
    f_rand = rng.normal(0, 1, 6)
    W = orc.weights(u, Nk, f_rand)
    # sum_k N_k W_nk = 1 for every sample and any f
    assert np.max(np.abs(W @ Nk - 1.0)) < 1e-13
    f, _ = orc.solve_mbar(u, Nk)
    W = orc.weights(u, Nk, f)
    colsum = W.sum(axis=0)
    sampled = Nk > 0
    assert np.max(np.abs(colsum[sampled] - 1.0)) < 1e-12
    H = orc.hessian(u, Nk, f_rand)
    assert np.max(np.abs(H - H.T)) < 1e-12 * np.abs(H).max()
    assert np.max(np.abs(H.sum(axis=1))) < 1e-10 * np.abs(H).max()
    ev = np.linalg.eigvalsh(H)
    assert ev.min() > -1e-9 * np.abs(ev).max()


@pytest.mark.parametrize("seed", range(3))
def test_p5_decimal_brute_force(orc, seed):
    g = np.random.default_rng(100 + seed)
    K = 2 + seed
    Nk = g.integers(1, 4, size=K)
    N = int(Nk.sum())
    u = g.normal(0, 1.5, size=(K, N))
    f, info = orc.solve_mbar(u, Nk)
    fb = brute.mbar_decimal(u.tolist(), Nk.tolist())
    assert np.max(np.abs(f - np.array(fb))) < 1e-13


def test_p5_decimal_with_unsampled_state(orc):
    g = np.random.default_rng(7)
    Nk = np.array([3, 0, 4, 2])
    u = g.normal(0, 1.0, size=(4, 9))
    f, info = orc.solve_mbar(u, Nk)
    fb = brute.mbar_decimal(u.tolist(), Nk.tolist())
    assert np.max(np.abs(f - np.array(fb))) < 1e-13


def test_p6_invariances(orc):
    p = synth.harmonic_1d(K=5, Nk=[60, 40, 70, 50, 30], seed=5)
    u, Nk = p["u"], p["Nk"]
    f, _ = orc.solve_mbar(u, Nk)
    rng = np.random.default_rng(1)
    c_n = rng.normal(0, 5, u.shape[1])
    f2, _ = orc.solve_mbar(u + c_n[None, :], Nk)
    assert np.max(np.abs(f2 - f)) < 1e-12
    a_k = rng.normal(0, 5, u.shape[0])
    f3, _ = orc.solve_mbar(u + a_k[:, None], Nk)
    expect = f + a_k - a_k[0]
    assert np.max(np.abs(f3 - expect)) < 1e-12
    perm_n = rng.permutation(u.shape[1])
    f4, _ = orc.solve_mbar(u[:, perm_n], Nk)
    assert np.max(np.abs(f4 - f)) < 1e-12
    perm_k = np.array([0, 3, 1, 4, 2])
    f5, _ = orc.solve_mbar(u[perm_k], Nk[perm_k])
    assert np.max(np.abs(f5 - f[perm_k])) < 1e-12


def test_p7_special_cases(orc):
    g = np.random.default_rng(2)
    u = g.normal(0, 2, size=(1, 37))
    f, _ = orc.solve_mbar(u, [37])
    assert f[0] == 0.0
    W = orc.weights(u, [37], f)
    # K = 1: W_n = exp(-u_n) / sum_m exp(-u_m) / ... equals 1/N only when f is the solution
    assert np.max(np.abs(W[:, 0] * 37 - 1.0)) < 1e-14
    row = g.normal(0, 2, size=50)
    u = np.tile(row, (4, 1))
    Nk = np.array([10, 15, 5, 20])
    f, _ = orc.solve_mbar(u, Nk)
    assert np.max(np.abs(f)) < 1e-14
    W = orc.weights(u, Nk, f)
    assert np.max(np.abs(W - 1.0 / 50)) < 1e-15


def test_p8_binned_equals_unbinned_on_expanded_data(orc):
    g = np.random.default_rng(3)
    K, P = 4, 9
    ubar = g.normal(0, 1, size=(K, P))
    H = g.integers(1, 6, size=P)
    Nk = np.array([int(H.sum()) - 3 * (K - 1)] + [3] * (K - 1))
    f = g.normal(0, 0.5, K)
    f_b = orc.sci_step(ubar, Nk, f, logH=np.log(H))
    u_exp = np.repeat(ubar, H, axis=1)
    f_u = orc.sci_step(u_exp, Nk, f)
    assert np.max(np.abs(f_b - f_u)) < 1e-13


def test_p8_unique_bins_mean_representative(orc):
    # with m = 1 and all quantised values distinct, MEAN bins are the samples
    p = synth.harmonic_1d(K=3, Nk=40, seed=4)
    q, lo, sc = orc.quantize(p["xi"])
    assert len(np.unique(q[:, 0])) == q.shape[0]
    cells, H, sb = orc.histogram(q, 1)
    assert np.all(H == 1)
    ub = orc.represent(3, 1, 1, lo, sc, cells, H, sample_bin=sb, u=p["u"])
    f = np.array([0.0, 0.3, -0.2])
    f_b = orc.sci_step(ub, p["Nk"], f, logH=np.log(H))
    f_u = orc.sci_step(p["u"], p["Nk"], f)
    assert np.max(np.abs(f_b - f_u)) < 1e-13


@pytest.mark.parametrize("d", [1, 2])
def test_p8_mean_representative_with_populated_bins(orc, d):
    # MEAN representative of a bin holding several samples: (1 / H_p) sum over
    # the bin's members of u_kn (the bin value in Eq. (1) for plain u_kn).
    # The bins are rebuilt here with numpy alone (cell = q // m per dimension,
    # ascending distinct cells) and the means taken by np.add.reduceat over
    # the samples sorted by bin, so a missing / H_p, a wrong member set or a
    # transposed K x P result fails.
    g = np.random.Generator(np.random.PCG64(40 + d))
    N, K = 3000, 5
    xi = g.normal(0.0, 1.0, size=(N, d))
    u = g.normal(0.0, 2.0, size=(K, N)) + 3.0 * np.arange(K)[:, None]
    q, lo, sc = orc.quantize(xi)
    m = 2**27 if d == 1 else 2**28
    qm = (q.astype(np.uint64) // np.uint64(m))
    if d == 1:
        cell = qm[:, 0]
    else:
        stride = np.uint64((2**32 - 1) // m + 1)
        cell = qm[:, 0] + qm[:, 1] * stride
    ucells, sb_np, H_np = np.unique(cell, return_inverse=True, return_counts=True)
    assert H_np.max() > 1 and len(ucells) > 10
    cells, H, sb = orc.histogram(q, m)
    assert np.array_equal(cells, ucells) and np.array_equal(H, H_np)
    assert np.array_equal(sb, sb_np.astype(np.int32))
    order = np.argsort(sb_np, kind="stable")
    starts = np.concatenate([[0], np.cumsum(H_np)[:-1]])
    ref = np.add.reduceat(u[:, order], starts, axis=1) / H_np[None, :]
    ub = orc.represent(K, d, m, lo, sc, cells, H, sample_bin=sb, u=u)
    assert ub.shape == (K, len(ucells))
    assert np.max(np.abs(ub - ref)) < 1e-12


def test_p8_centre_representative_is_model_at_centre(orc):
    # LINEAR model: the representative of a bin is the model at the bin centre,
    # which for a linear model equals the mean of the bin's lower and upper edge values.
    xi = np.array([[0.0], [1.0], [2.5], [10.0]])
    q, lo, sc = orc.quantize(xi)
    m = 2**31
    cells, H, sb = orc.histogram(q, m)
    coef = np.array([[1.0, 2.0, 0.0]])
    ub = orc.represent(1, 1, m, lo, sc, cells, H, model_type=1, coef=coef)
    width = m / sc[0]
    for p, c in enumerate(cells):
        left = lo[0] + c * width
        assert abs(ub[0, p] - (1.0 + 2.0 * (left + 0.5 * width))) < 1e-12


def _np_cells(q, m):
    q = q.astype(np.uint64)
    m = np.uint64(m)
    if q.shape[1] == 1:
        return q[:, 0] // m
    stride = np.uint64(4294967295) // m + np.uint64(1)
    return q[:, 0] // m + (q[:, 1] // m) * stride


@pytest.mark.parametrize("d", [1, 2])
def test_p9_binning_brute_force(orc, d):
    g = np.random.default_rng(20 + d)
    xi = g.normal(0, 1, size=(3000, d))
    xi[:50] = xi[50:100]  # duplicates
    q, lo, sc = orc.quantize(xi)
    # quantisation anchors: minimum -> 0, maximum -> 2^32 - 1, order preserved
    for j in range(d):
        assert q[np.argmin(xi[:, j]), j] == 0
        # (hi - lo) * ((2^32 - 1) / (hi - lo)) may round just below 2^32 - 1
        assert q[np.argmax(xi[:, j]), j] >= 4294967294
        o = np.argsort(xi[:, j], kind="stable")
        assert np.all(np.diff(q[o, j].astype(np.int64)) >= 0)
    for m in [1, 7, 1000, 123456, 2**20 + 3, 2**31, 2**32 - 1]:
        assert orc.nonempty_bins(q, m) == len(np.unique(_np_cells(q, m)))
    for n in [2, 10, 100, 1000, 2500]:
        m, gm, probes = orc.width_search(q, n)
        assert gm == len(np.unique(_np_cells(q, m)))
        if len(np.unique(_np_cells(q, 1))) < n:
            assert m == 1
        else:
            # bisection end state: g(m) >= n > g(m + 1)
            assert gm >= n
            assert len(np.unique(_np_cells(q, m + 1))) < n
        cells, H, sb = orc.histogram(q, m)
        uc, cnt = np.unique(_np_cells(q, m), return_counts=True)
        assert np.array_equal(cells, uc.astype(np.uint64))
        assert np.array_equal(H, cnt)
        assert np.array_equal(cells[sb], _np_cells(q, m))


def test_p9_width_search_exhaustive_small_range(orc):
    # small integer coordinates: for every target n, scan all widths and check
    # the bisection answer is a valid end state and matches a direct walk.
    xi = np.array([[v] for v in [0, 1, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144, 233]], float)
    q, lo, sc = orc.quantize(xi)
    for n in range(2, 15):
        m, gm, _ = orc.width_search(q, n)
        assert orc.nonempty_bins(q, m) == gm
        if gm >= n:
            assert orc.nonempty_bins(q, m + 1) < n


def test_p10_hessian_vs_finite_differences(orc):
    p = synth.harmonic_1d(K=4, Nk=[30, 20, 25, 35], seed=8)
    u, Nk = p["u"], p["Nk"]
    f = np.array([0.0, 0.2, -0.4, 0.1])
    H = orc.hessian(u, Nk, f)
    h = 1e-5
    for j in range(4):
        e = np.zeros(4)
        e[j] = h
        _, gp = orc.objective_gradient(u, Nk, f + e)
        _, gm = orc.objective_gradient(u, Nk, f - e)
        fd = (gp - gm) / (2 * h)
        assert np.max(np.abs(fd - H[:, j])) < 1e-6 * max(1.0, np.abs(H).max())
    # and the gradient is the derivative of the objective
    for j in range(4):
        e = np.zeros(4)
        e[j] = h
        Fp, _ = orc.objective_gradient(u, Nk, f + e)
        Fm, _ = orc.objective_gradient(u, Nk, f - e)
        _, g0 = orc.objective_gradient(u, Nk, f)
        assert abs((Fp - Fm) / (2 * h) - g0[j]) < 1e-6 * max(1.0, np.abs(g0).max())


def test_p11_fixed_point_certificate(orc):
    p = synth.double_well(K=20, Nk=500, seed=3)
    f, info = orc.solve_mbar(p["u"], p["Nk"])
    assert info["rc"] == 0
    assert info["residual"] < 1e-12
    _, g = orc.objective_gradient(p["u"], p["Nk"], f)
    assert np.max(np.abs(g / p["Nk"])) < 1e-12


def test_log_denominator_definition(orc):
    # ln D_n against a direct evaluation with N_k = 0 states excluded
    g = np.random.default_rng(9)
    u = g.normal(0, 1, size=(3, 11))
    Nk = np.array([5, 0, 6])
    f = np.array([0.0, 4.0, -1.0])
    ld = orc.log_denominator(u, Nk, f)
    direct = np.log(5 * np.exp(f[0] - u[0]) + 6 * np.exp(f[2] - u[2]))
    assert np.max(np.abs(ld - direct)) < 1e-14


def test_relative_step_eq2(orc):
    assert orc.rel_step([0.0, 2.0, -3.0], [0.0, 1.0, -2.0]) == pytest.approx(1.0)
    assert orc.rel_step([0.0, 1.0], [0.0, 0.0]) == math.inf
    assert orc.rel_step([5.0, 0.0], [1.0, 0.0]) == 0.0  # gauge state excluded


def test_reweight_equals_weights_of_sampled_state(orc):
    # At the solution, reweighting to a sampled state k gives p_n = W_nk
    # (Eqs. (5)-(6) with C the sum of the unnormalised terms).
    p = synth.harmonic_1d(K=4, Nk=200, seed=6)
    u, Nk = p["u"], p["Nk"]
    f, _ = orc.solve_mbar(u, Nk)
    ld = orc.log_denominator(u, Nk, f)
    W = orc.weights(u, Nk, f)
    for k in range(4):
        pk = orc.reweight(u[k], ld)
        assert abs(pk.sum() - 1.0) < 1e-14
        assert np.max(np.abs(pk - W[:, k])) < 1e-14


def test_bumbar_reaches_unbinned_solution(orc):
    p = synth.double_well(K=30, Nk=700, seed=5)
    f_ref, _ = orc.solve_mbar(p["u"], p["Nk"])
    f, info = orc.bumbar(p["u"], p["Nk"], p["xi"], p["model_type"], p["coef"], tol=1e-11)
    assert info["rc"] == 0
    assert np.max(np.abs(f - f_ref)) < 1e-10
    # schedule structure: decisions follow Eq. (3) on the reported steps,
    # and the loop stops exactly when 2 inc n exceeds N
    N = p["N"]
    n = 1000
    for c in info["checks"]:
        assert c["n"] == n
        same = c["P"] == c["P_next"]
        assert c["refine"] == int(2 * c["s_next"] > 10 * c["s_n"] or same) or same
        if c["refine"]:
            n *= 10
        assert c["stop"] == int(bool(c["refine"]) and 2 * 10 * n > N)
    assert info["checks"][-1]["stop"] == 1


def test_bumbar_replay_reproduces_schedule(orc):
    p = synth.double_well(K=20, Nk=600, seed=6)
    f, info = orc.bumbar(p["u"], p["Nk"], p["xi"], p["model_type"], p["coef"])
    flags = [c["refine"] for c in info["checks"]]
    f2, info2 = orc.bumbar(p["u"], p["Nk"], p["xi"], p["model_type"], p["coef"],
                           replay=(info["phase1"], flags))
    assert np.array_equal(info2["f_binned"], info["f_binned"])
    assert [c["refine"] for c in info2["checks"]] == flags


def test_bumbar_mean_representatives_2d(orc):
    p = synth.ladder_2d(K=12, Nk=300, seed=1)
    f_ref, _ = orc.solve_mbar(p["u"], p["Nk"])
    f, info = orc.bumbar(p["u"], p["Nk"], p["xi"], model_type=0, coef=None, tol=1e-11)
    assert info["rc"] == 0
    assert np.max(np.abs(f - f_ref)) < 1e-9
    f2, info2 = orc.bumbar(p["u"], p["Nk"], p["xi"], p["model_type"], p["coef"], tol=1e-11)
    assert np.max(np.abs(f2 - f_ref)) < 1e-9


def test_pmf_uniform_weights_are_histogram_counts(orc):
    # With p_n = 1/N the surface is -ln of the normalised histogram. Samples
    # sit at least 1e-6 of a bin away from every edge, so no rounding of the
    # bin formula can move one; bins on the sides stay empty (+inf).
    g = np.random.default_rng(3)
    nb, lo, hi = 40, -2.0, 3.0
    w = (hi - lo) / nb
    cells = g.integers(5, 35, 20000)
    x = lo + (cells + g.uniform(1e-6, 1 - 1e-6, cells.size)) * w
    p = np.full(x.size, 1.0 / x.size)
    F = orc.pmf(x, p, lo, hi, nb)
    counts = np.bincount(cells, minlength=nb)
    for b in range(nb):
        if counts[b]:
            assert F[b] == pytest.approx(-math.log(counts[b] / x.size), rel=1e-13)
        else:
            assert F[b] == math.inf
    hist, _ = np.histogram(x, bins=nb, range=(lo, hi), weights=p)
    ok = hist > 0
    assert np.allclose(np.exp(-F[ok]), hist[ok], rtol=1e-13, atol=0)


def test_pmf_2d_row_major_and_weighted(orc):
    # Unequal bin counts per axis, so a transposed index or swapped axis
    # fails; weights differ per sample, so a dropped p_n fails.
    g = np.random.default_rng(4)
    nb = (7, 5)
    lo, hi = (0.0, -1.0), (7.0, 4.0)
    i = g.integers(0, nb[0], 5000)
    j = g.integers(0, nb[1], 5000)
    x = np.stack([i + g.uniform(0.01, 0.99, i.size), j - 1.0 + g.uniform(0.01, 0.99, j.size)], 1)
    p = g.uniform(0.1, 1.0, i.size)
    F = orc.pmf(x, p, lo, hi, nb)
    assert F.shape == nb
    for a in range(nb[0]):
        for b in range(nb[1]):
            s = p[(i == a) & (j == b)].sum()
            assert F[a, b] == pytest.approx(-math.log(s), rel=1e-12)
    H, _, _ = np.histogram2d(x[:, 0], x[:, 1], bins=nb, range=[[0, 7], [-1, 4]], weights=p)
    assert np.allclose(np.exp(-F), H, rtol=1e-12, atol=0)


def test_pmf_edges_and_outside_samples(orc):
    # x = lo is in the first bin, x = hi and anything past either end is left
    # out; a bin whose samples all carry p = 0 has F = +inf.
    x = np.array([0.0, 0.5, 0.999, 1.0, -0.1, 2.0, 0.25])
    p = np.array([0.1, 0.2, 0.3, 0.9, 0.9, 0.9, 0.0])
    F = orc.pmf(x, p, 0.0, 1.0, 4)
    assert F[0] == pytest.approx(-math.log(0.1))
    assert F[1] == math.inf  # only the p = 0 sample
    assert F[2] == pytest.approx(-math.log(0.2))
    assert F[3] == pytest.approx(-math.log(0.3))
    with pytest.raises(RuntimeError):
        orc.pmf(x, p, 1.0, 1.0, 4)
    with pytest.raises(RuntimeError):
        orc.pmf(x, p, 0.0, 1.0, 0)


def test_pmf_of_reweighted_samples_is_target_potential(orc):
    # Samples of the state u_0 = x^2 / 2 (standard normal) reweighted to
    # u_1 = (x - 1/2)^2 / 2 with the one-state solution (logD_n = -u_0,n up to
    # a constant, removed by the normalisation of Eqs. (5)-(6)); the surface
    # then approaches u_1 plus a constant where the bins are well sampled.
    g = np.random.default_rng(11)
    x = g.normal(0.0, 1.0, 2_000_000)
    u0, u1 = 0.5 * x ** 2, 0.5 * (x - 0.5) ** 2
    p = orc.reweight(u1, -u0)
    nb, lo, hi = 20, -1.0, 1.5
    F = orc.pmf(x, p, lo, hi, nb)
    c = lo + (np.arange(nb) + 0.5) * (hi - lo) / nb
    ref = 0.5 * (c - 0.5) ** 2
    shift = np.mean(F - ref)
    assert np.max(np.abs(F - ref - shift)) < 0.02
