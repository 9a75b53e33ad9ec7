"""Batches of binned SCI steps replayed as HIP graphs against the same kernels
launched one by one (option graphs = 0): the solve must give the same bits.

Every replay writes the relative steps of its steps, and the stage decides
from them, so equal schedules (every check's s values and refine flags), equal
iteration counts and an equal f mean every replay matched the eager launches.
Between replays the stage runs its own eager copies and readbacks on the same
stream. Cases: stored bin representatives (1-D), the FP64 model at the bin
centres (2-D, on the fly), the FP32 model at the centres (K > 256, mixed
precision), and a context on a non-default stream.
"""
import sys

import numpy as np
import pytest

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
    import paper_2609_03541_amd as bm
    return bm


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x)).cuda()


def schedule(info):
    return [(c["n"], c["P"], c["P_next"], c["s_n"], c["s_next"], c["refine"], c["stop"])
            for c in info["checks"]]


def same_solve(bm, args, kw, batched=None):
    f1, i1 = bm.solve(*args, graphs=1, **kw)
    f0, i0 = bm.solve(*args, graphs=0, **kw)
    say("  graph batches", i1["graph_batches"], "phase1", i1["phase1_iters"], "phase2",
        i1["phase2_iters"], "checks", i1["n_checks"], "single-workgroup steps",
        i1["batched_steps"])
    # the first level (at most 128 bins here) runs in single-workgroup batches
    # whenever its matrix is stored in FP64
    if batched is not None:
        assert (i1["batched_steps"] > 0) == batched
        assert i1["batched_steps"] == i0["batched_steps"]
    assert i1["status"] == i0["status"] == 0
    assert i0["graph_batches"] == 0
    # each replay is a batch: a stage of several levels replays some shapes
    assert i1["graph_batches"] > i1["n_checks"] // 2
    assert i1["phase1_iters"] == i0["phase1_iters"]
    assert i1["phase2_iters"] == i0["phase2_iters"]
    assert schedule(i1) == schedule(i0)
    assert np.array_equal(f1.cpu().numpy(), f0.cpu().numpy())


def test_graphs_stored_representatives(bm):
    p = synth.double_well(K=30, Nk=700, seed=5)
    say(f"stored u, 1-D: K={p['K']} N={p['N']}")
    same_solve(bm, (dev(p["u"]), p["Nk"]),
               dict(xi=p["xi"], model=p["model_type"], coef=p["coef"], tol=1e-11), batched=True)


def test_graphs_model_fp64_centres(bm):
    p = synth.double_well(K=40, Nk=800, seed=9)
    say(f"on the fly, FP64 centres: K={p['K']} N={p['N']}")
    same_solve(bm, (None, p["Nk"]),
               dict(xi=p["xi"], model=p["model_type"], coef=p["coef"], tol=1e-11), batched=True)


def test_graphs_model_fp32_centres(bm):
    p = synth.ladder_2d(K=300, Nk=40, seed=6)
    say(f"on the fly, mixed precision: K={p['K']} N={p['N']}")
    same_solve(bm, (None, p["Nk"]),
               dict(xi=p["xi"], model=p["model_type"], coef=p["coef"], precision=1, tol=1e-11),
               batched=False)


def test_graphs_on_a_side_stream(bm):
    import torch
    p = synth.double_well(K=20, Nk=500, seed=12)
    say(f"side stream: K={p['K']} N={p['N']}")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        u = dev(p["u"])
        same_solve(bm, (u, p["Nk"]),
                   dict(xi=p["xi"], model=p["model_type"], coef=p["coef"], tol=1e-11))
    torch.cuda.synchronize()
