"""GPU tests of batched serving and of the on-device model energies.

A served problem must give bitwise the result of the same problem solved
alone (same kernels and launch shapes, deterministic reductions), and the
FP64 oracle's solution to 1e-9 kT. Admission is checked through the
server's counters: with room for several problems they run concurrently;
with an arena that holds one at a time they run one after another.
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


def small_stream(n, seed=11):
    specs = synth.serving_stream(n_problems=n, seed=seed, K_range=(3, 24), Nk_range=(40, 300))
    return [synth.materialize_problem(s) for _, s in specs]


def test_model_energies_match_generator(bm):
    say("model energies: harmonic 2-D and linear 2-D")
    p = synth.muller_brown_grid(G=5, Nk=60, seed=4, materialize=True)
    u = bm.model_energies(p["xi"], p["coef"], p["model_type"], p["K"]).cpu().numpy()
    assert u.shape == p["u"].shape
    assert np.max(np.abs(u - p["u"]) / (1.0 + np.abs(p["u"]))) < 1e-13
    q = synth.ladder_2d(K=20, Nk=50, seed=2)
    u2 = bm.model_energies(q["xi"], q["coef"], q["model_type"], q["K"]).cpu().numpy()
    assert np.max(np.abs(u2 - q["u"]) / (1.0 + np.abs(q["u"]))) < 1e-13
    h = synth.harmonic_1d(K=6, Nk=100, seed=3)
    u3 = bm.model_energies(h["xi"][:, 0], h["coef"], h["model_type"], h["K"]).cpu().numpy()
    assert np.max(np.abs(u3 - h["u"]) / (1.0 + np.abs(h["u"]))) < 1e-13


def test_model_energies_reject_bad_arguments(bm):
    p = synth.harmonic_1d(K=4, Nk=10, seed=0)
    with pytest.raises(bm.BumbarError):
        bm.model_energies(p["xi"], p["coef"], bm.MODEL_NONE, p["K"])
    with pytest.raises(bm.BumbarError):
        bm.model_energies(np.zeros((10, 3)), np.zeros((4, 7)), bm.MODEL_LINEAR, 4)


def test_served_results_equal_solo_and_oracle(bm):
    probs = small_stream(10)
    srv = bm.Server(hbm_budget_bytes=1 << 30, max_active=4)
    try:
        tickets = []
        for i, p in enumerate(probs):
            binning = i % 3 != 2  # a mix of BU-MBAR and plain MBAR requests
            tickets.append(srv.submit(p["Nk"], u=p["u"], xi=p["xi"], model=p["model_type"],
                                      coef=p["coef"], binning=binning, tol=1e-11))
        for i, (p, t) in enumerate(zip(probs, tickets)):
            say(f"served problem {i}: K={p['K']} N={p['N']}")
            f, info = srv.result(t)
            assert info["status"] == 0
            binning = i % 3 != 2
            f_solo, _ = bm.solve(dev(p["u"]), p["Nk"], xi=p["xi"], model=p["model_type"],
                                 coef=p["coef"], binning=binning, tol=1e-11)
            assert np.array_equal(f, f_solo.cpu().numpy()), i
            f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
            assert np.max(np.abs(f - f_ref)) < 1e-9, i
            assert info["latency_ms"] > 0
        c = srv.counters()
        assert c["completed"] == len(probs)
        assert c["peak_active"] >= 2
        assert 0 < c["peak_bytes"] <= 1 << 30
    finally:
        srv.close()


def test_model_request_solved_on_the_fly(bm):
    p = synth.muller_brown_grid(G=6, Nk=150, seed=4, materialize=True)
    say(f"model-only request K={p['K']} N={p['N']}")
    srv = bm.Server(hbm_budget_bytes=1 << 28, max_active=2)
    try:
        t = srv.submit(p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"], tol=1e-11)
        srv.wait(t)
        assert srv.poll(t) == 2  # BUMBAR_TICKET_DONE
        f, info = srv.result(t)
        assert info["status"] == 0
        with pytest.raises(bm.BumbarError):
            srv.poll(t)  # a result is read once; the ticket is then released
    finally:
        srv.close()
    f_solo, _ = bm.solve(None, p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                         tol=1e-11)
    assert np.array_equal(f, f_solo.cpu().numpy())
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    assert np.max(np.abs(f - f_ref)) < 1e-9


def footprint_bound(bm, K, N, d, binning):
    ctx = bm.context()
    # the same options the server's request carries (bin-centre representatives)
    opts = bm.default_options(binning=int(binning), represent=bm.REPRESENT_CENTRE)
    ws = ctx.query_workspace(K, N, d if binning else 0, opts)
    parts = [8 * K * N, 8 * N * d, 8 * K, 8 * K * (1 + 2 * d), 8 * K, ws]
    return sum(-(-b // 256) * 256 for b in parts)


def test_admission_by_footprint(bm):
    p = synth.harmonic_1d(K=16, Nk=2000, seed=9)
    fp = footprint_bound(bm, p["K"], p["N"], 1, True)
    # room for one resident problem at a time: four slots, but no overlap
    srv = bm.Server(hbm_budget_bytes=int(fp * 1.5), max_active=4)
    try:
        ts = [srv.submit(p["Nk"], u=p["u"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                         tol=1e-11) for _ in range(4)]
        fs = [srv.result(t)[0] for t in ts]
        c = srv.counters()
        say("tight arena counters", c)
        assert c["peak_active"] == 1
        assert c["peak_bytes"] <= fp * 1.5
        for f in fs[1:]:
            assert np.array_equal(f, fs[0])
        with pytest.raises(bm.BumbarError) as e:
            big = synth.harmonic_1d(K=16, Nk=20000, seed=9)
            srv.submit(big["Nk"], u=big["u"], tol=1e-11)
        assert e.value.code == bm.ETOOBIG
    finally:
        srv.close()


def test_failed_request_reports_status(bm):
    p = synth.harmonic_1d(K=4, Nk=100, seed=1)
    srv = bm.Server(hbm_budget_bytes=1 << 26, max_active=2)
    try:
        bad = srv.submit(p["Nk"], u=p["u"], tol=0.0)  # rejected by the solve's host checks
        good = srv.submit(p["Nk"], u=p["u"], tol=1e-11)
        f, info = srv.result(bad)
        assert info["status"] == bm.EINVAL
        assert srv.poll(good) in (0, 1, 2)
        f2, info2 = srv.result(good)
        assert info2["status"] == 0
        f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
        assert np.max(np.abs(f2 - f_ref)) < 1e-9
    finally:
        srv.close()


def test_mixed_precision_served_equals_solo(bm):
    # mixed precision in the mix: each served result is bitwise the result of
    # the same mixed solve alone, and within 1e-6 kT of the oracle
    specs = synth.serving_stream(n_problems=8, seed=21, K_range=(40, 120), Nk_range=(200, 600))
    probs = [synth.materialize_problem(s) for _, s in specs]
    srv = bm.Server(hbm_budget_bytes=1 << 30, max_active=4)
    try:
        ts = [srv.submit(p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"], tol=1e-10,
                         precision=bm.PREC_MIXED) for p in probs]
        for i, (p, t) in enumerate(zip(probs, ts)):
            f, info = srv.result(t)
            say(f"mixed served problem {i}: K={p['K']} N={p['N']} status={info['status']}")
            assert info["status"] == 0
            f_solo, info_solo = bm.solve(None, p["Nk"], xi=p["xi"], model=p["model_type"],
                                         coef=p["coef"], tol=1e-10, precision=bm.PREC_MIXED)
            assert np.array_equal(f, f_solo.cpu().numpy()), i
            f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
            assert np.max(np.abs(f - f_ref)) < 1e-6, i
        assert srv.counters()["peak_active"] >= 2
    finally:
        srv.close()
