"""The temperature ladder shaped like the paper's parallel-tempering example
(Section 4: 50 temperatures spaced geometrically over a factor of two, unit-
variance energies at 80% neighbour overlap), solved three ways on the GPU:
BU-MBAR (bins on E, the LINEAR model at the bin centres, Newton finisher),
plain SCI, and plain Newton (one SCI step, then Newton).

At N_k = 2000 every variant is held to 1e-9 kT of the oracle's certified
solution. At the paper's N_k = 2e5 (N = 1e7, u 4 GB in FP64, built on the
device) BU-MBAR and plain Newton agree to 1e-9 kT and the oracle's fixed-
point residual at the BU-MBAR result is below 1e-9 kT.
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


def variants(bm, xi, coef):
    return {
        "bumbar": dict(xi=xi, model=bm.MODEL_LINEAR, coef=coef),
        "newton": dict(binning=False, finisher=bm.FINISH_NEWTON, sci_switch=1e300),
        "sci": dict(binning=False, finisher=bm.FINISH_SCI, max_iter=200000),
    }


def test_ladder_three_ways_small(bm):
    p = synth.temperature_ladder(K=50, Nk=2000, seed=3)
    say(f"temperature ladder K={p['K']} N={p['N']}")
    f_ref, inf = oracle.solve_mbar(p["u"], p["Nk"])
    assert inf["rc"] == 0
    u = dev(p["u"])
    for name, kw in variants(bm, p["xi"], p["coef"]).items():
        f, info = bm.solve(u, p["Nk"], tol=1e-11, **kw)
        err = np.max(np.abs(f.cpu().numpy() - f_ref))
        say(f"  {name}: status {info['status']} binned {info['phase1_iters'] + info['phase2_iters']}"
            f" finisher {info['finisher_steps']} err {err:.2e}")
        assert info["status"] == 0
        assert err < 1e-9


def test_ladder_full_size(bm):
    import torch
    p = synth.temperature_ladder(K=50, Nk=200000, seed=3, materialize=False)
    K, N = p["K"], p["N"]
    say(f"temperature ladder full size K={K} N={N}")
    xi, coef = dev(p["xi"]), dev(p["coef"])
    u = bm.model_energies(xi, coef, bm.MODEL_LINEAR, K)
    out = {}
    for name in ("bumbar", "newton"):
        f, info = bm.solve(u, p["Nk"], tol=1e-10, **variants(bm, xi, coef)[name])
        say(f"  {name}: status {info['status']} finisher {info['finisher_steps']} "
            f"grad {info['grad_norm']:.2e}")
        assert info["status"] == 0
        out[name] = f.cpu().numpy()
    assert np.max(np.abs(out["bumbar"] - out["newton"])) < 1e-9
    del u
    torch.cuda.empty_cache()
    uh = p["beta"][:, None] * p["xi"][:, 0][None, :]
    res = np.max(np.abs(oracle.sci_step(uh, p["Nk"], out["bumbar"]) - out["bumbar"]))
    say(f"  oracle fixed-point residual at the BU-MBAR result: {res:.3e}")
    assert res < 1e-9
