"""The replica-count study (Section 4, Fig. 3) against the oracle, 12 seeds.

Temperature ladders of M replicas with unit-variance energy histograms at
80% neighbour overlap and N_k = N0 / M^p per replica (scenarios i, ii, iii:
p = 0, 1, 2). tests/golden holds the oracle's certified f for every seed of
every point with N0 scaled by 1/100 (N0 = 1e2, 3e4, 9e6; 144 problems) and
for the full-size points with M^2 N_k <= 3e7 (36 problems). Each problem is
solved on the GPU by BU-MBAR and by plain Newton; both must reach the
oracle's f to 1e-9 kT.
"""
import json
import os
import sys
from collections import defaultdict

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def groups():
    out = defaultdict(list)
    for name in ("fig3_replicas_reduced", "fig3_replicas_full_small"):
        path = os.path.join(GOLDEN, name + ".json")
        if not os.path.exists(path):
            continue
        with open(path) as fh:
            g = json.load(fh)
        for it in g["problems"]:
            out[(name, it["scenario"], it["M"])].append(it)
    return sorted(out.items(), key=lambda kv: (kv[0][0], kv[0][1], kv[0][2]))


GROUPS = groups()


@pytest.fixture(scope="module")
def bm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_03541_amd as bm
    return bm


def test_golden_covers_the_study():
    # 12 seeds at every point of the reduced study, and the full-size points
    names = defaultdict(int)
    for (name, _, _), items in GROUPS:
        names[name] += len(items)
        assert len(items) == 12
    assert names["fig3_replicas_reduced"] == 144
    assert names["fig3_replicas_full_small"] == 36


@pytest.mark.parametrize("key,items", GROUPS, ids=[f"{k[0][12:]}-{k[1]}-M{k[2]}" for k, _ in GROUPS])
def test_replica_study_matches_oracle(bm, key, items):
    import torch
    name, scen, M = key
    worst = 0.0
    for it in items:
        assert it["certificate"]["sci_residual"] < 1e-10
        p = synth.temperature_ladder(K=M, Nk=it["Nk"], seed=it["seed"], materialize=False)
        xi = torch.tensor(p["xi"], device="cuda")
        coef = torch.tensor(p["coef"], device="cuda")
        u = bm.model_energies(xi, coef, bm.MODEL_LINEAR, M)
        g = np.asarray(it["f"])
        fb, ib = bm.solve(u, p["Nk"], xi=xi, model=bm.MODEL_LINEAR, coef=coef, tol=1e-10)
        fn, inn = bm.solve(u, p["Nk"], binning=False, sci_switch=1e300, tol=1e-10)
        assert ib["status"] == 0 and inn["status"] == 0, it["seed"]
        e = max(float(np.max(np.abs(fb.cpu().numpy() - g))),
                float(np.max(np.abs(fn.cpu().numpy() - g))))
        worst = max(worst, e)
        assert e < 1e-9, (it["seed"], e)
    say(f"{name} scenario {scen} M={M}: 12 seeds, worst error {worst:.2e} kT")
