"""GPU tests of the cooperative batches of binned steps.

A batch of binned self-consistent steps (Eq. (1) with the bin counts,
Algorithm 1) on a level held in the sample-major layout (256 < K <= 1024)
runs as one cooperative launch. Its steps must give the schedule of the
per-step kernels (sweep, partial sums, finaliser): the same phase-1 length,
the same checks (n, bins, refine decisions), the same relative steps to
1e-9, and a final f within 1e-10 kT of theirs and 1e-9 kT of the FP64
oracle's fixed point.
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


# K = 1000 (rows of 1024) is checked against the per-step kernels only: the
# oracle's certified solve takes minutes there (the full-size ladder at
# K = 1000 is held to the oracle's golden f by test_gpu_golden)
@pytest.mark.parametrize("K,Nk,seed,check_oracle", [(300, 100, 5, True), (520, 60, 6, True),
                                                    (1000, 40, 7, False)])
def test_cooperative_batches_match_per_step_kernels(bm, K, Nk, seed, check_oracle):
    import torch
    p = synth.ladder_2d(K=K, Nk=Nk, seed=seed)
    u = torch.tensor(p["u"], device="cuda")
    kw = dict(xi=p["xi"], model=p["model_type"], coef=p["coef"], tol=1e-11)
    say(f"K={K} N={p['N']}: cooperative batches")
    f1, i1 = bm.solve(u, p["Nk"], grid_batches=1, **kw)
    say(f"K={K}: per-step kernels")
    f0, i0 = bm.solve(u, p["Nk"], grid_batches=0, **kw)
    say(f"coop_steps {i1['coop_steps']} phase1 {i1['phase1_iters']}/{i0['phase1_iters']} "
        f"checks {i1['n_checks']}/{i0['n_checks']}")
    assert i1["status"] == 0 and i0["status"] == 0
    assert i1["coop_steps"] > 0 and i0["coop_steps"] == 0
    assert i1["phase1_iters"] == i0["phase1_iters"]
    key = [(c["n"], c["P"], c["P_next"], c["refine"], c["stop"]) for c in i1["checks"]]
    assert key == [(c["n"], c["P"], c["P_next"], c["refine"], c["stop"]) for c in i0["checks"]]
    for a, b in zip(i1["checks"], i0["checks"]):
        for name in ("s_n", "s_next"):
            assert abs(a[name] - b[name]) <= 1e-9 * max(abs(b[name]), 1e-300), (name, a, b)
    f1n, f0n = f1.cpu().numpy(), f0.cpu().numpy()
    assert np.max(np.abs(f1n - f0n)) < 1e-10
    if check_oracle:
        f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
        assert np.max(np.abs(f1n - f_ref)) < 1e-9


def test_cooperative_batches_with_unsampled_states(bm):
    # states with N_k = 0 are left out of D (the masked sweep) and get f from
    # the MBAR formula: both forms agree
    import torch
    p = synth.ladder_2d(K=400, Nk=80, seed=8)
    Nk = np.array(p["Nk"]).copy()
    keep = np.ones(p["N"], dtype=bool)
    # drop the samples of every 7th state (N_k = 0 there)
    starts = np.concatenate([[0], np.cumsum(Nk)[:-1]])
    for k in range(3, 400, 7):
        keep[starts[k]:starts[k] + Nk[k]] = False
        Nk[k] = 0
    u_np = np.ascontiguousarray(p["u"][:, keep])
    xi = np.ascontiguousarray(p["xi"][keep])
    u = torch.tensor(u_np, device="cuda")
    kw = dict(xi=xi, model=p["model_type"], coef=p["coef"], tol=1e-11)
    f1, i1 = bm.solve(u, Nk, grid_batches=1, **kw)
    f0, i0 = bm.solve(u, Nk, grid_batches=0, **kw)
    say(f"unsampled: coop_steps {i1['coop_steps']}")
    assert i1["status"] == 0 and i0["status"] == 0 and i1["coop_steps"] > 0
    assert i1["phase1_iters"] == i0["phase1_iters"] and i1["n_checks"] == i0["n_checks"]
    assert np.max(np.abs(f1.cpu().numpy() - f0.cpu().numpy())) < 1e-10
    f_ref, _ = oracle.solve_mbar(u_np, Nk)
    assert np.max(np.abs(f1.cpu().numpy() - f_ref)) < 1e-9
