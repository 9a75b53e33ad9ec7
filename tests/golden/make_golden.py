"""Write the golden free energies of the full-size workloads, from the oracle only.

Each golden f is the FP64 CPU oracle's certified MBAR solution (Section 2:
the binned iteration converges to the unbinned equations), computed here
with no input from the GPU library:
  1. Algorithm 1 as the oracle runs it (oracle.bumbar: binned stage, then a
     short unbinned SCI stage), from f = 0;
  2. Newton polish on the unbinned objective: the gradient, the line search
     and the stopping test are the oracle's compensated C sums; the Hessian
     H = diag(S) - P^T P (P_nk = N_k W_nk, the weights from oracle.weights)
     is accumulated over sample chunks with a numpy matrix product, a library
     primitive standing in for the oracle's plain loops, which would take
     days at K = 1000, N = 2e6 (it only shapes the steps);
  3. certification: the full Newton step below 1e-13 kT and the fixed-point
     residual max |SCI(f) - f| below 1e-12 kT, both recorded.

Usage: python tests/golden/make_golden.py {c0,c1,c2,tladder,c4r,c3sub,fig3r,fig3} ...
Inputs are the seeded generators of synth (the same recipes the GPU tests and
the benchmark use). Output: tests/golden/<name>.json.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def say(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def hessian_chunked(u, Nk, f, chunk):
    K, N = u.shape
    H = np.zeros((K, K))
    S = np.zeros(K)
    for n0 in range(0, N, chunk):
        W = oracle.weights(np.ascontiguousarray(u[:, n0:n0 + chunk]), Nk, f)
        P = W * Nk[None, :].astype(np.float64)
        S += P.sum(axis=0)
        H -= P.T @ P
    H[np.diag_indices(K)] += S
    return H


def certify(u, Nk, f, chunk=100_000, max_steps=40):
    """Newton polish (oracle gradient and line search) to a certified fixed point."""
    f = np.asarray(f, dtype=np.float64).copy()
    f -= f[0]
    _, g = oracle.objective_gradient(u, Nk, f)
    gn = np.linalg.norm(g)
    steps = 0
    full_step = np.inf
    for steps in range(1, max_steps + 1):
        H = hessian_chunked(u, Nk, f, chunk)
        d = oracle.newton_direction(Nk, H, g)
        if d is None:
            raise RuntimeError("reduced Hessian not positive definite")
        full_step = float(np.max(np.abs(d)))
        if full_step < 1e-12:
            # rounding floor of the gradient: the full step itself bounds the
            # remaining distance; take it and stop
            f = f + d
            f -= f[0]
            say(f"  newton {steps}: |g| {gn:.3e} full step {full_step:.3e} (floor)")
            break
        alpha, accepted = 1.0, False
        for _ in range(31):
            ft = f + alpha * d
            ft -= ft[0]
            _, g2 = oracle.objective_gradient(u, Nk, ft)
            if np.linalg.norm(g2) < gn:
                accepted = True
                break
            alpha *= 0.5
        say(f"  newton {steps}: |g| {gn:.3e} full step {full_step:.3e} alpha {alpha:g}")
        if not accepted:
            # at the rounding floor the gradient norm stops falling
            break
        f, g, gn = ft, g2, np.linalg.norm(g2)
        if alpha == 1.0 and full_step < 1e-13:
            break
    res = float(np.max(np.abs(oracle.sci_step(u, Nk, f) - f)))
    say(f"  certified: newton steps {steps}, last full step {full_step:.3e}, residual {res:.3e}")
    return f, dict(newton_steps=steps, last_full_step=full_step, sci_residual=res,
                   grad_norm=float(gn))


def solve_golden(u, Nk, xi, model, coef, tol_sci=1e-3, chunk=100_000):
    t0 = time.time()
    fb, info = oracle.bumbar(u, Nk, xi, model, coef, tol=tol_sci, finisher=1)
    say(f"  Algorithm 1: phase1 {info['phase1']} phase2 {info['phase2']} checks "
        f"{info['n_checks']} sci {info['finisher_steps']} ({time.time() - t0:.0f} s)")
    f, cert = certify(u, Nk, fb, chunk=chunk)
    cert.update(algorithm1=dict(phase1=info["phase1"], phase2=info["phase2"],
                                n_checks=info["n_checks"], sci=info["finisher_steps"]),
                oracle_seconds=time.time() - t0)
    return f, cert


def write(name, recipe, f, cert, extra=None):
    out = dict(name=name, recipe=recipe, f=[float(v) for v in f], certificate=cert,
               threads=os.cpu_count(), made_by="tests/golden/make_golden.py (oracle and synth only)")
    if extra:
        out.update(extra)
    path = os.path.join(HERE, name + ".json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    say("wrote", path)


def ladder_u(p):
    E, V = p["xi"][:, 0], p["xi"][:, 1]
    K = len(p["beta"])
    u = np.empty((K, len(E)))
    for k in range(K):
        u[k] = p["beta"][k] * E + p["lam"][k] * V
    return u


def run_c2():
    # temperature / alchemical ladder, K = 1000, N_k = 2000 (N = 2e6), seed 2
    p = synth.ladder_2d(K=1000, Nk=2000, seed=2, materialize=False)
    u = ladder_u(p)
    say("c2 ladder_2d K=1000 N=2e6: u", u.nbytes / 1e9, "GB")
    f, cert = solve_golden(u, p["Nk"], p["xi"], p["model_type"], p["coef"])
    write("c2_ladder_K1000_N2e6", "synth.ladder_2d(K=1000, Nk=2000, seed=2); u = beta E + lambda V",
          f, cert)


def run_tladder():
    p = synth.temperature_ladder(K=50, Nk=200_000, seed=3)
    say("temperature ladder K=50 N=1e7")
    f, cert = solve_golden(p["u"], p["Nk"], p["xi"], p["model_type"], p["coef"], chunk=1_000_000)
    write("tladder_K50_N1e7", "synth.temperature_ladder(K=50, Nk=200000, seed=3)", f, cert)


def run_c4r():
    # Muller-Brown 40 x 40 umbrella grid with N_k reduced to 500 (N = 8e5) so
    # that u fits the host: u_kn = kappa/2 |r_n - c_k|^2 from the FP32 coordinates
    p = synth.muller_brown_grid(G=40, Nk=500, seed=4, materialize=True)
    say("c4 reduced: K=1600 N=8e5")
    f, cert = solve_golden(p["u"], p["Nk"], p["xi"], p["model_type"], p["coef"], chunk=50_000)
    write("c4r_mullerbrown_K1600_N8e5", "synth.muller_brown_grid(G=40, Nk=500, seed=4)", f, cert)


def run_c0():
    p = synth.harmonic_1d(K=8, Nk=1000, seed=0)
    f, cert = solve_golden(p["u"], p["Nk"], p["xi"], p["model_type"], p["coef"])
    # the analytic free energies of the wells (beta = 1): f_k - f_0 = ln(kappa_k / kappa_0) / 2
    analytic = 0.5 * np.log(p["kappa"] / p["kappa"][0])
    write("c0_harmonic_K8_N8e3", "synth.harmonic_1d(K=8, Nk=1000, seed=0)", f, cert,
          extra=dict(analytic=[float(v) for v in analytic]))


def run_c1():
    # double-well umbrella sampling, K = 100 windows, N_k = 1e4 (N = 1e6), seed 1
    p = synth.double_well(K=100, Nk=10000, seed=1)
    say("c1 double well K=100 N=1e6")
    f, cert = solve_golden(p["u"], p["Nk"], p["xi"], p["model_type"], p["coef"], chunk=200_000)
    write("c1_double_well_K100_N1e6", "synth.double_well(K=100, Nk=10000, seed=1)", f, cert)


def run_c3sub():
    # every 8th problem of the 512-problem serving stream (seed 3): 64 problems
    stream = synth.serving_stream(n_problems=512, seed=3)
    items = []
    for j in range(0, 512, 8):
        t, spec = stream[j]
        p = synth.materialize_problem(spec, materialize=True)
        say(f"c3 problem {j}: {spec['kind']} K={p['K']} N={p['N']}")
        f, cert = solve_golden(p["u"], p["Nk"], p["xi"], p["model_type"], p["coef"],
                               chunk=200_000)
        sp = dict(kind=spec["kind"], K=int(spec["K"]), Nk=[int(v) for v in spec["Nk"]],
                  seed=int(spec["seed"]))
        items.append(dict(index=j, spec=sp, f=[float(v) for v in f], certificate=cert))
        del p
    path = os.path.join(HERE, "c3_stream_subset64.json")
    with open(path, "w") as fh:
        json.dump(dict(name="c3_stream_subset64",
                       recipe="synth.serving_stream(n_problems=512, seed=3), problems 0, 8, ..., 504",
                       problems=items, threads=os.cpu_count(),
                       made_by="tests/golden/make_golden.py (oracle and synth only)"), fh)
    say("wrote", path)


# The replica-count study of Section 4 (Fig. 3): temperature ladders of M
# replicas with unit-variance energy histograms at 80% neighbour overlap and
# N_k = N0 / M^p per replica, scenario i (p = 0, N0 = 1e4), ii (p = 1,
# N0 = 3e6), iii (p = 2, N0 = 9e8), M in {10, 30, 100, 300}, 12 seeds each.
FIG3_SCENARIOS = (("i", 1e4, 0), ("ii", 3e6, 1), ("iii", 9e8, 2))
FIG3_M = (10, 30, 100, 300)


def fig3_seed(M, si, s):
    return 9000 + 100 * M + 10 * si + s


def fig3_problems(scale):
    """(scenario, M, N_k, seed) of the study with every N0 multiplied by scale."""
    out = []
    for si, (name, n0, pw) in enumerate(FIG3_SCENARIOS):
        for M in FIG3_M:
            nk = int(round(n0 * scale / M ** pw))
            for s in range(12):
                out.append((name, M, nk, fig3_seed(M, si, s)))
    return out


def run_fig3(scale, name, max_elems):
    items = []
    for scen, M, nk, seed in fig3_problems(scale):
        if M * M * nk > max_elems:
            continue
        p = synth.temperature_ladder(K=M, Nk=nk, seed=seed)
        say(f"fig3 {scen} M={M} N_k={nk} seed={seed}")
        f, cert = solve_golden(p["u"], p["Nk"], p["xi"], p["model_type"], p["coef"],
                               chunk=200_000)
        items.append(dict(scenario=scen, M=M, Nk=nk, seed=seed, f=[float(v) for v in f],
                          certificate=cert))
    path = os.path.join(HERE, name + ".json")
    with open(path, "w") as fh:
        json.dump(dict(name=name,
                       recipe=f"synth.temperature_ladder(K=M, Nk=round(N0 * {scale:g} / M^p), "
                              f"seed=9000 + 100 M + 10 scenario + s), s = 0..11, "
                              f"M * M * Nk <= {max_elems:g}",
                       problems=items, threads=os.cpu_count(),
                       made_by="tests/golden/make_golden.py (oracle and synth only)"), fh)
    say("wrote", path)


if __name__ == "__main__":
    oracle.build()
    jobs = dict(c0=run_c0, c1=run_c1, c2=run_c2, tladder=run_tladder, c4r=run_c4r, c3sub=run_c3sub,
                fig3r=lambda: run_fig3(0.01, "fig3_replicas_reduced", 1e12),
                fig3=lambda: run_fig3(1.0, "fig3_replicas_full_small", 3e7))
    for name in sys.argv[1:] or list(jobs):
        jobs[name]()
