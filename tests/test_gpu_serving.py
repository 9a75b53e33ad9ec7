"""GPU tests of batched serving and of the on-device model energies.

A served problem must give bitwise the result of the same problem solved
alone (same kernels and launch shapes, deterministic reductions), and the
FP64 oracle's solution to 1e-9 kT. Admission is checked through the
server's counters: with room for several problems they run concurrently;
with an arena that holds one at a time they run one after another. Both
ways of driving the slots (worker threads, and caller-driven fibers that
advance only inside progress()) give the same bits.
"""
import sys
import time

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
        assert c["mem_waits"] >= 1  # slots were free, memory was not
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


def test_caller_driven_server_advances_only_in_progress(bm):
    # no worker threads: nothing is admitted or run between progress() calls;
    # driven by progress() alone the results are bitwise those of the solo
    # solves and of a threaded server
    probs = small_stream(8, seed=13)
    kw = [dict(u=p["u"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
               binning=i % 3 != 2, tol=1e-11) for i, p in enumerate(probs)]
    srv = bm.Server(hbm_budget_bytes=1 << 30, max_active=3, caller_driven=True)
    try:
        ts = [srv.submit(p["Nk"], **k) for p, k in zip(probs, kw)]
        time.sleep(0.3)
        assert [srv.poll(t) for t in ts] == [0] * len(ts)  # all still QUEUED
        done = srv.progress()
        states = [srv.poll(t) for t in ts]
        say("after one tick", states, "done", done)
        assert all(s in (1, 2) for s in states[:3]) and states[3:] == [0] * 5
        ticks, t0 = 1, time.time()
        while done < len(ts):
            done += srv.progress()
            ticks += 1
            assert time.time() - t0 < 60, "caller-driven server made no progress"
        say("ticks", ticks)
        res = [srv.result(t, wait=False) for t in ts]
        c = srv.counters()
        assert c["completed"] == len(ts) and c["peak_active"] == 3
    finally:
        srv.close()
    thr = bm.Server(hbm_budget_bytes=1 << 30, max_active=3)
    try:
        tt = [thr.submit(p["Nk"], **k) for p, k in zip(probs, kw)]
        res_thr = [thr.result(t) for t in tt]
    finally:
        thr.close()
    for i, (p, k) in enumerate(zip(probs, kw)):
        f, info = res[i]
        assert info["status"] == 0 and info["latency_ms"] > 0
        assert np.array_equal(f, res_thr[i][0]), i
        kk = dict(k)
        f_solo, _ = bm.solve(dev(kk.pop("u")), p["Nk"], **kk)
        assert np.array_equal(f, f_solo.cpu().numpy()), i


def test_caller_driven_wait_and_close_drive_the_fibers(bm):
    # wait() ticks until its ticket is done; close() runs the admitted solves
    # to the end and fails the queued ones
    probs = small_stream(5, seed=17)
    srv = bm.Server(hbm_budget_bytes=1 << 30, max_active=2, caller_driven=True)
    ts = [srv.submit(p["Nk"], u=p["u"], tol=1e-11) for p in probs]
    f, info = srv.result(ts[3])  # waits: tickets 0-2 are admitted and run first
    assert info["status"] == 0
    f_solo, _ = bm.solve(dev(probs[3]["u"]), probs[3]["Nk"], tol=1e-11)
    assert np.array_equal(f, f_solo.cpu().numpy())
    srv.close()


@pytest.mark.parametrize("caller_driven", [False, True])
def test_materialized_fp32_requests(bm, caller_driven):
    # u evaluated once on the device from the model and stored in FP32 (4 B
    # per element in the footprint), solved in mixed precision as a stored
    # FP32 matrix: bitwise the solo solve of that matrix, and the oracle's
    # solution of the FP32-rounded problem to 1e-9 kT
    import torch
    specs = synth.serving_stream(n_problems=4, seed=23, K_range=(40, 120), Nk_range=(200, 600))
    probs = [synth.materialize_problem(s) for _, s in specs]
    srv = bm.Server(hbm_budget_bytes=1 << 30, max_active=3, caller_driven=caller_driven)
    try:
        ts = [srv.submit(p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                         materialize=True, tol=1e-10, precision=bm.PREC_MIXED) for p in probs]
        res = [srv.result(t) for t in ts]
    finally:
        srv.close()
    for i, (p, (f, info)) in enumerate(zip(probs, res)):
        say(f"materialised FP32 problem {i}: K={p['K']} N={p['N']} status={info['status']}")
        assert info["status"] == 0 and info["mixed_steps"] >= 1
        u32 = bm.model_energies(p["xi"], p["coef"], p["model_type"], p["K"], dtype=torch.float32)
        f_solo, _ = bm.solve(u32, p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                             tol=1e-10, precision=bm.PREC_MIXED)
        assert np.array_equal(f, f_solo.cpu().numpy()), i
        f_ref, _ = oracle.solve_mbar(u32.double().cpu().numpy(), p["Nk"])
        assert np.max(np.abs(f - f_ref)) < 1e-9, i


@pytest.mark.parametrize("kind", ["fp64_stored", "fp32_materialized"])
def test_fused_server_equals_solo_and_oracle(bm, kind):
    # a fusing server gathers the small binned batches of all its problems
    # into one graph-replayed launch per tick; every result is bitwise the
    # solo solve's (same code per item) and the oracle's to the tolerance
    import torch
    if kind == "fp64_stored":
        probs = small_stream(12, seed=31)
        kw = [dict(u=p["u"], xi=p["xi"], model=p["model_type"], coef=p["coef"], tol=1e-11)
              for p in probs]
    else:
        specs = synth.serving_stream(n_problems=8, seed=37, K_range=(20, 120),
                                     Nk_range=(200, 600))
        probs = [synth.materialize_problem(s) for _, s in specs]
        kw = [dict(xi=p["xi"], model=p["model_type"], coef=p["coef"], materialize=True,
                   tol=1e-10, precision=bm.PREC_MIXED) for p in probs]
    srv = bm.Server(hbm_budget_bytes=1 << 30, max_active=6, caller_driven=True, fuse=True)
    try:
        ts = [srv.submit(p["Nk"], **k) for p, k in zip(probs, kw)]
        res = [srv.result(t) for t in ts]
        c = srv.counters()
    finally:
        srv.close()
    say(f"fused {kind}: {c['fused_launches']} launches, {c['fused_items']} batches")
    assert c["fused_launches"] >= 1 and c["fused_items"] > c["fused_launches"]
    for i, (p, k, (f, info)) in enumerate(zip(probs, kw, res)):
        say(f"fused {kind} problem {i}: K={p['K']} N={p['N']} status={info['status']} "
            f"batched={info['batched_steps']}")
        assert info["status"] == 0
        kk = dict(k)
        if kind == "fp64_stored":
            f_solo, _ = bm.solve(dev(kk.pop("u")), p["Nk"], **kk)
            f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
        else:
            kk.pop("materialize")
            u32 = bm.model_energies(p["xi"], p["coef"], p["model_type"], p["K"],
                                    dtype=torch.float32)
            f_solo, _ = bm.solve(u32, p["Nk"], **kk)
            f_ref, _ = oracle.solve_mbar(u32.double().cpu().numpy(), p["Nk"])
        assert np.array_equal(f, f_solo.cpu().numpy()), i
        assert np.max(np.abs(f - f_ref)) < 1e-9, i
