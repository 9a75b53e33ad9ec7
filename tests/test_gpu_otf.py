"""GPU parity of the on-the-fly path (u_kn evaluated from the bias model inside
the kernels) against the FP64 oracle fed the materialised u_kn.

FP64 model kernels: single sweeps and Hessians to 1e-12 (as for a stored
FP64 matrix), full solves to 1e-9 kT. FP32 model kernels (mixed precision):
single sweeps to 2e-4 kT, the level FP32 evaluation of the expanded
quadratic in log2 units reaches for energies of a few tens of kT; solves
that end with the FP64 refinement to 1e-9 kT.
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


def aniso_2d(K, Nk, seed, unsampled=()):
    """2-D harmonic windows with per-axis force constants; u from the model definition."""
    g = np.random.default_rng(seed)
    cx, cy = g.uniform(-1.5, 1.5, K), g.uniform(-1.0, 1.0, K)
    kx, ky = g.uniform(4, 30, K), g.uniform(4, 30, K)
    a = g.uniform(-1, 1, K)
    counts = np.full(K, Nk, dtype=np.int64)
    for k in unsampled:
        counts[k] = 0
    owner = np.repeat(np.arange(K), counts)
    x = g.normal(cx[owner], 1 / np.sqrt(kx[owner]))
    y = g.normal(cy[owner], 1 / np.sqrt(ky[owner]))
    xi = np.stack([x, y], axis=1)
    coef = np.stack([a, kx, cx, ky, cy], axis=1)
    u = (a[:, None] + 0.5 * kx[:, None] * (x[None, :] - cx[:, None]) ** 2
         + 0.5 * ky[:, None] * (y[None, :] - cy[:, None]) ** 2)
    return dict(u=u, Nk=counts, xi=xi, coef=coef, model_type=synth.MODEL_HARMONIC, K=K,
                N=int(counts.sum()))


def grid_2d(nx, ny, Nk, seed, unsampled=(), span=1.5, kappa=(8.0, 30.0), a_far=0.0):
    """Windows on an nx x ny product grid: per-column kx and centre, per-row ky
    and centre, a per-state constant a_k (a_far added to every state but the
    first); u from the model definition."""
    g = np.random.default_rng(seed)
    gx, gy = np.linspace(-span, span, nx), np.linspace(-span, span, ny)
    kxs, kys = g.uniform(*kappa, nx), g.uniform(*kappa, ny)
    ix, iy = np.tile(np.arange(nx), ny), np.repeat(np.arange(ny), nx)
    K = nx * ny
    cx, cy, kx, ky = gx[ix], gy[iy], kxs[ix], kys[iy]
    a = g.uniform(-1, 1, K)
    a[1:] += a_far
    counts = np.full(K, Nk, dtype=np.int64)
    for k in unsampled:
        counts[k] = 0
    owner = np.repeat(np.arange(K), counts)
    x = g.normal(cx[owner], 1 / np.sqrt(kx[owner]))
    y = g.normal(cy[owner], 1 / np.sqrt(ky[owner]))
    coef = np.stack([a, kx, cx, ky, cy], axis=1)
    u = (a[:, None] + 0.5 * kx[:, None] * (x[None, :] - cx[:, None]) ** 2
         + 0.5 * ky[:, None] * (y[None, :] - cy[:, None]) ** 2)
    return dict(u=u, Nk=counts, xi=np.stack([x, y], axis=1), coef=coef,
                model_type=synth.MODEL_HARMONIC, K=K, N=int(counts.sum()))


def cases():
    return {
        "harmonic_1d": lambda: synth.harmonic_1d(K=8, Nk=1000, seed=0),
        "harmonic_1d_K700": lambda: synth.harmonic_1d(K=700, Nk=9, seed=5),
        "aniso_2d": lambda: aniso_2d(K=37, Nk=131, seed=3),
        "aniso_2d_unsampled": lambda: aniso_2d(K=20, Nk=157, seed=4, unsampled=(0, 7)),
        "linear_2d": lambda: synth.ladder_2d(K=30, Nk=77, seed=2),
        "muller_brown": lambda: synth.muller_brown_grid(G=5, Nk=60, seed=4, materialize=True),
        # product grids with 4 (Ix + Jy) <= K: the FP64 sweeps take the factored passes
        "muller_brown_grid12": lambda: synth.muller_brown_grid(G=12, Nk=30, seed=7,
                                                               materialize=True),
        "aniso_grid": lambda: grid_2d(10, 12, 25, seed=11, unsampled=(3, 50, 119)),
    }


def start_point(p, seed=1):
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    g = np.random.default_rng(seed)
    f = f_ref + g.normal(0, 0.05, p["K"])
    return f - f[0]


@pytest.mark.parametrize("name", list(cases()))
def test_model_sweep_fp64_matches_oracle(bm, name):
    p = cases()[name]()
    say(f"model sweep FP64 {name}: K={p['K']} N={p['N']}")
    f = start_point(p)
    fn_ref, lD_ref = oracle.sci_step(p["u"], p["Nk"], f, return_logD=True)
    fn, lD, S, st = bm.sweep_model(p["xi"], p["coef"], p["model_type"], p["Nk"], f)
    fn, lD, S = fn.cpu().numpy(), lD.cpu().numpy(), S.cpu().numpy()
    assert np.max(np.abs(lD - lD_ref)) < 1e-12 * max(1.0, np.abs(lD_ref).max())
    assert np.max(np.abs(fn - fn_ref)) < 1e-11
    W = oracle.weights(p["u"], p["Nk"], f)
    S_ref = p["Nk"] * W.sum(axis=0)
    samp = p["Nk"] > 0
    assert np.max(np.abs(S[samp] - S_ref[samp]) / S_ref[samp]) < 1e-11
    F_ref, g_ref = oracle.objective_gradient(p["u"], p["Nk"], f)
    assert abs(st["objective"] - F_ref) < 1e-10 * max(1.0, abs(F_ref))


@pytest.mark.parametrize("name", list(cases()))
def test_model_sweep_fp32_close_to_oracle(bm, name):
    p = cases()[name]()
    say(f"model sweep FP32 {name}: K={p['K']} N={p['N']}")
    f = start_point(p)
    fn_ref, lD_ref = oracle.sci_step(p["u"], p["Nk"], f, return_logD=True)
    fn, lD, S, st = bm.sweep_model(p["xi"], p["coef"], p["model_type"], p["Nk"], f,
                                   precision=bm.PREC_MIXED)
    assert np.max(np.abs(lD.cpu().numpy() - lD_ref)) < 2e-4
    assert np.max(np.abs(fn.cpu().numpy() - fn_ref)) < 2e-4


@pytest.mark.parametrize("name", ["harmonic_1d", "aniso_2d_unsampled", "linear_2d",
                                  "harmonic_1d_K700"])
def test_model_hessian_matches_oracle(bm, name):
    p = cases()[name]()
    say(f"model hessian {name}: K={p['K']} N={p['N']}")
    f = start_point(p)
    H_ref = oracle.hessian(p["u"], p["Nk"], f)
    scale = np.abs(H_ref).max()
    _, lD, S, _ = bm.sweep_model(p["xi"], p["coef"], p["model_type"], p["Nk"], f)
    H = bm.hessian_model(p["xi"], p["coef"], p["model_type"], p["Nk"], f, lD, S).cpu().numpy()
    assert np.max(np.abs(H - H_ref)) < 1e-12 * scale
    H32 = bm.hessian_model(p["xi"], p["coef"], p["model_type"], p["Nk"], f, lD, S,
                           precision=bm.PREC_MIXED).cpu().numpy()
    assert np.max(np.abs(H32 - H_ref)) < 1e-3 * scale


@pytest.mark.parametrize("name,binning,precision", [
    ("harmonic_1d", False, 0), ("harmonic_1d", True, 0), ("aniso_2d", True, 0),
    ("aniso_2d_unsampled", True, 1), ("linear_2d", True, 1), ("muller_brown", True, 1),
    ("harmonic_1d_K700", True, 1)])
def test_solve_on_the_fly_matches_oracle(bm, name, binning, precision):
    p = cases()[name]()
    say(f"on-the-fly solve {name}: K={p['K']} N={p['N']} binning={binning} prec={precision}")
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    f, info = bm.solve(None, p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                       binning=binning, precision=precision, tol=1e-11, want_weights=True,
                       want_logD=True)
    assert info["status"] == 0
    fh = f.cpu().numpy()
    assert np.max(np.abs(fh - f_ref)) < 1e-9
    lD_ref = oracle.log_denominator(p["u"], p["Nk"], fh)
    assert np.max(np.abs(info["logD"].cpu().numpy() - lD_ref)) < 1e-12 * max(1, np.abs(lD_ref).max())
    W_ref = oracle.weights(p["u"], p["Nk"], fh)
    assert np.max(np.abs(info["W"].cpu().numpy() - W_ref)) < 1e-12
    if precision == 1:
        say("  mixed steps", info["mixed_steps"], "newton", info["finisher_steps"])


def test_mixed_on_the_fly_large_energies(bm):
    # K > 256 on the fly in mixed precision: the binned steps start on the
    # FP32 model sweep (falling back to FP64 if FP32 rounding of these large
    # ladder energies stalls its step tests); the result is the FP64 one
    p = synth.ladder_2d(K=300, Nk=40, seed=6)
    say(f"mixed on-the-fly ladder: K={p['K']} N={p['N']}")
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    f, info = bm.solve(None, p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                       precision=1, tol=1e-11)
    assert info["status"] == 0
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9


def test_on_the_fly_equals_stored_solve(bm):
    # the same problem with u stored and u from the model reaches the same f
    p = aniso_2d(K=25, Nk=200, seed=8)
    f1, _ = bm.solve(dev(p["u"]), p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                     tol=1e-12)
    f2, _ = bm.solve(None, p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"], tol=1e-12)
    assert np.max(np.abs(f1.cpu().numpy() - f2.cpu().numpy())) < 1e-10


def test_on_the_fly_rejects_missing_model(bm):
    p = synth.harmonic_1d(K=4, Nk=50, seed=1)
    with pytest.raises(ValueError):
        bm.solve(None, p["Nk"], xi=p["xi"])
    with pytest.raises(bm.BumbarError):
        bm.sweep_model(p["xi"], p["coef"], bm.MODEL_NONE, p["Nk"], np.zeros(4))


def test_grid_sweep_far_offsets(bm):
    # every state but one 660 kT up, sweep from f = 0: most samples' factored
    # column sums fall below 1e-280 and take the direct sum over the states,
    # and the state pass carries weights near 1e286
    p = grid_2d(12, 12, 20, seed=13, span=4.0, kappa=(25.0, 30.0), a_far=660.0)
    say(f"grid sweep, far offsets: K={p['K']} N={p['N']}")
    f = np.zeros(p["K"])
    fn_ref, lD_ref = oracle.sci_step(p["u"], p["Nk"], f, return_logD=True)
    fn, lD, S, st = bm.sweep_model(p["xi"], p["coef"], p["model_type"], p["Nk"], f)
    fn, lD, S = fn.cpu().numpy(), lD.cpu().numpy(), S.cpu().numpy()
    assert np.max(np.abs(lD - lD_ref)) < 1e-12 * max(1.0, np.abs(lD_ref).max())
    assert np.max(np.abs(fn - fn_ref)) < 1e-12 * max(1.0, np.abs(fn_ref).max())
    W = oracle.weights(p["u"], p["Nk"], f)
    S_ref = p["Nk"] * W.sum(axis=0)
    assert np.max(np.abs(S - S_ref) / S_ref) < 1e-11


@pytest.mark.parametrize("precision", [0, 1])
def test_grid_solve_uses_factored_sweeps(bm, precision):
    p = grid_2d(12, 10, 60, seed=17, unsampled=(7,))
    say(f"grid solve precision={precision}: K={p['K']} N={p['N']}")
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    f, info = bm.solve(None, p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                       precision=precision, tol=1e-11)
    say("  grid sweeps", info["grid_sweeps"], "unbinned sweeps", info["unbinned_sweeps"])
    assert info["status"] == 0
    assert info["grid_sweeps"] > 0
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9


def test_grid_mixed_large_k(bm):
    # K > 256 on a product grid in mixed precision: binned steps and Newton
    # sweeps on the factored FP64 passes, Hessian from the FP32 model on the
    # matrix cores; the result is the FP64 one
    p = synth.muller_brown_grid(G=17, Nk=12, seed=9, materialize=True)
    say(f"grid mixed K={p['K']} N={p['N']}")
    f_ref, _ = oracle.solve_mbar(p["u"], p["Nk"])
    f, info = bm.solve(None, p["Nk"], xi=p["xi"], model=p["model_type"], coef=p["coef"],
                       precision=1, tol=1e-11)
    say("  grid sweeps", info["grid_sweeps"], "hessians", info["hessians"])
    assert info["status"] == 0
    assert info["grid_sweeps"] > 0
    assert np.max(np.abs(f.cpu().numpy() - f_ref)) < 1e-9
