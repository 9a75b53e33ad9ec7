"""Seeded synthetic MBAR inputs (numpy only).

This module builds the inputs both the GPU solver and the CPU oracle are run
on: reduced energies u_kn, per-state sample counts N_k, the binning
coordinates xi and the reduced-energy model (for bin-centre representatives
and for energies computed on the fly). It holds none of the MBAR arithmetic
(no log-sum-exp, no free energies); it only draws samples and evaluates the
bias potentials that define each synthetic workload.

Workloads (shapes follow the paper's examples: temperature ladders with
unit-variance normal energies at 80% neighbour overlap, Section 4, and
sample sets of 1e4-1e7 points, Sections 3-4):

* ``harmonic_1d``      K harmonic wells, exact Gaussian draws (analytic f).
* ``double_well``      1-D umbrella sampling of U(x) = (x^2 - 1)^2 with
                       Metropolis chains.
* ``ladder_2d``        temperature/alchemical ladder u_kn = beta_k E_n + lambda_k V_n.
* ``temperature_ladder`` the shape of the paper's parallel-tempering example
                       (Section 4): K = 50 temperatures spaced geometrically
                       over a factor of two, u_kn = beta_k E_n, unit-variance
                       energies at 80% neighbour overlap.
* ``muller_brown_grid`` 2-D umbrella grid on a scaled Muller-Brown surface.
* ``serving_stream``   a Poisson stream of independent small problems.

Model coefficient layout (per state, stride 1 + 2d):
  LINEAR   u_k(x) = c_k + sum_j a_kj x_j            -> [c_k, a_k1, ..., a_kd, 0...]
  HARMONIC u_k(x) = c_k + sum_j kappa_kj/2 (x_j - x0_kj)^2 -> [c_k, kappa_k1, x0_k1, ...]
"""
from __future__ import annotations

import math

import numpy as np

MODEL_NONE = 0
MODEL_LINEAR = 1
MODEL_HARMONIC = 2

# Mean spacing of two unit-variance normals whose overlap coefficient
# integral(min(p, q)) = 2 Phi(-delta / 2) equals 0.8 (80% neighbour overlap).
OVERLAP80_DELTA = 0.5066942


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _harmonic_u(x, kappa, x0):
    """u_kn = kappa_k / 2 (x_n - x0_k)^2 for 1-D samples x (N) -> K x N float64."""
    x = np.asarray(x, dtype=np.float64)
    dx = x[None, :] - np.asarray(x0, dtype=np.float64)[:, None]
    return 0.5 * np.asarray(kappa, dtype=np.float64)[:, None] * (dx * dx)


def _problem(u, Nk, xi, model_type, coef, **meta):
    out = dict(u=None if u is None else np.ascontiguousarray(u, dtype=np.float64),
               Nk=np.ascontiguousarray(Nk, dtype=np.int64),
               xi=np.ascontiguousarray(xi, dtype=np.float64),
               model_type=model_type,
               coef=np.ascontiguousarray(coef, dtype=np.float64))
    out["K"] = len(out["Nk"])
    out["N"] = int(out["Nk"].sum())
    out["d"] = out["xi"].shape[1]
    out.update(meta)
    return out


def harmonic_1d(K=8, Nk=1000, seed=0, kappa_range=(0.5, 4.0), x_range=(-2.0, 2.0),
                materialize=True):
    """K 1-D harmonic wells u_k(x) = kappa_k (x - x_k)^2 / 2 at beta = 1.

    kappa_k ~ U[0.5, 4] (all K drawn first), then x_k ~ U[-2, 2]; state k
    contributes Nk exact draws x ~ N(x_k, 1/sqrt(kappa_k)); samples are
    concatenated state by state. Nk may be an int or a length-K sequence.
    """
    g = _rng(seed)
    kappa = g.uniform(kappa_range[0], kappa_range[1], K)
    x0 = g.uniform(x_range[0], x_range[1], K)
    counts = np.full(K, Nk, dtype=np.int64) if np.isscalar(Nk) else np.asarray(Nk, np.int64)
    xs = [g.normal(x0[k], 1.0 / math.sqrt(kappa[k]), int(counts[k])) for k in range(K)]
    x = np.concatenate(xs) if len(xs) else np.zeros(0)
    u = _harmonic_u(x, kappa, x0) if materialize else None
    coef = np.zeros((K, 3))
    coef[:, 1] = kappa
    coef[:, 2] = x0
    return _problem(u, counts, x[:, None], MODEL_HARMONIC, coef, kappa=kappa, x0=x0,
                    name=f"harmonic_1d K={K} Nk={Nk}")


def double_well_potential(x):
    return (x * x - 1.0) ** 2


def double_well(K=100, Nk=10000, kappa=50.0, seed=1, burn=1000, thin=10, sigma=0.1,
                span=(-1.5, 1.5)):
    """Umbrella sampling of U(x) = (x^2 - 1)^2 at beta = 1.

    Window k has centre x_k = span[0] + (span[1] - span[0]) k / (K - 1) and
    bias kappa/2 (x - x_k)^2. Each window runs a Metropolis chain from x_k
    with Gaussian proposals of width sigma, discards ``burn`` steps and keeps
    every ``thin``-th state until it holds Nk samples. All chains advance in
    lock-step (one vectorised draw per step). u_kn = U(x_n) + kappa/2 (x_n - x_k)^2.
    """
    g = _rng(seed)
    xc = span[0] + (span[1] - span[0]) * np.arange(K) / max(K - 1, 1)

    def energy(x):
        return double_well_potential(x) + 0.5 * kappa * (x - xc) ** 2

    x = xc.copy()
    e = energy(x)
    out = np.empty((Nk, K))
    total = burn + thin * Nk
    kept = 0
    for step in range(1, total + 1):
        prop = x + sigma * g.standard_normal(K)
        ep = energy(prop)
        acc = np.log(g.random(K)) < (e - ep)
        x = np.where(acc, prop, x)
        e = np.where(acc, ep, e)
        if step > burn and (step - burn) % thin == 0:
            out[kept] = x
            kept += 1
    samples = out.T.reshape(-1)  # state-major concatenation
    u = double_well_potential(samples)[None, :] + _harmonic_u(samples, np.full(K, kappa), xc)
    coef = np.zeros((K, 3))
    coef[:, 1] = kappa
    coef[:, 2] = xc
    return _problem(u, np.full(K, Nk), samples[:, None], MODEL_HARMONIC, coef, centres=xc,
                    kappa=kappa, name=f"double_well K={K} Nk={Nk}")


def ladder_2d(K=1000, Nk=2000, seed=2, beta_range=(0.5, 2.0), delta=OVERLAP80_DELTA,
              materialize=True):
    """Temperature/alchemical ladder u_kn = beta_k E_n + lambda_k V_n.

    beta_k = b0 (b1/b0)^(k/(K-1)) (geometric), lambda_k = k/(K-1). State k
    contributes Nk samples with E ~ N(-delta k, 1) and V ~ N(-delta k / 2, 1),
    delta giving 80% overlap between neighbouring energy histograms.
    """
    g = _rng(seed)
    ks = np.arange(K)
    t = ks / max(K - 1, 1)
    beta = beta_range[0] * (beta_range[1] / beta_range[0]) ** t
    lam = t.astype(np.float64)
    E = np.concatenate([g.normal(-delta * k, 1.0, Nk) for k in range(K)])
    V = np.concatenate([g.normal(-delta * k / 2.0, 1.0, Nk) for k in range(K)])
    u = (beta[:, None] * E[None, :] + lam[:, None] * V[None, :]) if materialize else None
    coef = np.zeros((K, 5))
    coef[:, 1] = beta
    coef[:, 2] = lam
    xi = np.stack([E, V], axis=1)
    return _problem(u, np.full(K, Nk), xi, MODEL_LINEAR, coef, beta=beta, lam=lam,
                    name=f"ladder_2d K={K} Nk={Nk}")


def temperature_ladder(K=50, Nk=200000, seed=3, beta_range=(1.0, 2.0), delta=OVERLAP80_DELTA,
                       materialize=True):
    """Temperature ladder u_kn = beta_k E_n (1-D, LINEAR model on E).

    beta_k = b0 (b1/b0)^(k/(K-1)): temperatures geometric over a factor of
    b1/b0 = 2 (as 298 K to 600 K in the paper's replica set). State k draws
    Nk energies E ~ N(-delta k, 1), delta giving 80% overlap between
    neighbouring energy histograms.
    """
    g = _rng(seed)
    ks = np.arange(K)
    t = ks / max(K - 1, 1)
    beta = beta_range[0] * (beta_range[1] / beta_range[0]) ** t
    E = np.concatenate([g.normal(-delta * k, 1.0, Nk) for k in range(K)])
    u = (beta[:, None] * E[None, :]) if materialize else None
    coef = np.zeros((K, 3))
    coef[:, 1] = beta
    return _problem(u, np.full(K, Nk), E[:, None], MODEL_LINEAR, coef, beta=beta,
                    name=f"temperature_ladder K={K} Nk={Nk}")


# Muller-Brown potential (Muller & Brown, Theor. Chim. Acta 53, 75 (1979)).
_MB_A = np.array([-200.0, -100.0, -170.0, 15.0])
_MB_a = np.array([-1.0, -1.0, -6.5, 0.7])
_MB_b = np.array([0.0, 0.0, 11.0, 0.6])
_MB_c = np.array([-10.0, -10.0, -6.5, 0.7])
_MB_x0 = np.array([1.0, 0.0, -0.5, -1.0])
_MB_y0 = np.array([0.0, 0.5, 1.5, 1.0])


def muller_brown(x, y, scale=0.1):
    dx = x[..., None] - _MB_x0
    dy = y[..., None] - _MB_y0
    return scale * np.sum(_MB_A * np.exp(_MB_a * dx * dx + _MB_b * dx * dy + _MB_c * dy * dy),
                          axis=-1)


def muller_brown_grid(G=40, Nk=5000, kappa=20.0, seed=4, burn=1000, thin=5, sigma=0.1,
                      xr=(-1.5, 1.0), yr=(-0.5, 2.0), materialize=False):
    """2-D umbrella grid on the scaled (x0.1) Muller-Brown surface, beta = 1.

    G x G windows with centres on a uniform grid over xr x yr and isotropic
    bias kappa/2 |r - c_k|^2; Metropolis per window as in ``double_well``.
    Coordinates are stored as float32 (x, y). The common potential cancels in
    MBAR, so u_kn = kappa/2 |r_n - c_k|^2 evaluated from the float32
    coordinates (widened to float64) is the reduced energy.
    """
    g = _rng(seed)
    gx = xr[0] + (xr[1] - xr[0]) * np.arange(G) / max(G - 1, 1)
    gy = yr[0] + (yr[1] - yr[0]) * np.arange(G) / max(G - 1, 1)
    cx = np.tile(gx, G)      # state k = iy * G + ix
    cy = np.repeat(gy, G)
    K = G * G

    def energy(px, py):
        return muller_brown(px, py) + 0.5 * kappa * ((px - cx) ** 2 + (py - cy) ** 2)

    px, py = cx.copy(), cy.copy()
    e = energy(px, py)
    out = np.empty((Nk, K, 2), dtype=np.float32)
    total = burn + thin * Nk
    kept = 0
    for step in range(1, total + 1):
        qx = px + sigma * g.standard_normal(K)
        qy = py + sigma * g.standard_normal(K)
        eq = energy(qx, qy)
        acc = np.log(g.random(K)) < (e - eq)
        px = np.where(acc, qx, px)
        py = np.where(acc, qy, py)
        e = np.where(acc, eq, e)
        if step > burn and (step - burn) % thin == 0:
            out[kept, :, 0] = px
            out[kept, :, 1] = py
            kept += 1
    xy32 = np.ascontiguousarray(out.transpose(1, 0, 2).reshape(-1, 2))
    coef = np.zeros((K, 5))
    coef[:, 1] = kappa
    coef[:, 2] = cx
    coef[:, 3] = kappa
    coef[:, 4] = cy
    u = None
    if materialize:
        r = xy32.astype(np.float64)
        u = 0.5 * kappa * ((r[None, :, 0] - cx[:, None]) ** 2 + (r[None, :, 1] - cy[:, None]) ** 2)
    prob = _problem(u, np.full(K, Nk), xy32.astype(np.float64), MODEL_HARMONIC, coef,
                    name=f"muller_brown_grid {G}x{G} Nk={Nk}")
    prob["xi32"] = xy32
    return prob


def double_well_iid(K, Nk, kappa, seed, span=(-1.5, 1.5), grid=8192, materialize=True):
    """Independent draws from each biased double-well window by inverse CDF on a grid.

    Used for the serving stream, where running hundreds of Metropolis chains
    per problem would dominate generation time. ``Nk`` is a length-K array.
    """
    g = _rng(seed)
    xc = span[0] + (span[1] - span[0]) * np.arange(K) / max(K - 1, 1)
    lo, hi = span[0] - 1.0, span[1] + 1.0
    xs = np.linspace(lo, hi, grid)
    dxg = xs[1] - xs[0]
    parts = []
    for k in range(K):
        w = np.exp(-(double_well_potential(xs) + 0.5 * kappa * (xs - xc[k]) ** 2))
        cdf = np.cumsum(w)
        cdf /= cdf[-1]
        r = g.random(int(Nk[k]))
        idx = np.searchsorted(cdf, r)
        parts.append(xs[np.minimum(idx, grid - 1)] + (g.random(int(Nk[k])) - 0.5) * dxg)
    x = np.concatenate(parts)
    u = None
    if materialize:
        u = double_well_potential(x)[None, :] + _harmonic_u(x, np.full(K, kappa), xc)
    coef = np.zeros((K, 3))
    coef[:, 1] = kappa
    coef[:, 2] = xc
    return _problem(u, Nk, x[:, None], MODEL_HARMONIC, coef, name=f"double_well_iid K={K}")


def serving_stream(n_problems=512, seed=3, K_range=(4, 256), Nk_range=(100, 20000),
                   rate=None, materialize=False, max_K=None, max_Nk=None):
    """Seeded stream of independent MBAR problems for the batched server.

    Problem j: K_j ~ U{K_range}, N_kj ~ U{Nk_range} per state; even j =
    harmonic wells (``harmonic_1d`` recipe with K_j states), odd j = double-well
    windows with kappa = 50 ((K_j - 1)/99)^2 (i.i.d. inverse-CDF draws).
    Arrival times are cumulative exponential gaps at ``rate`` problems/s
    (None = all at t = 0). Returns a list of (arrival_time, problem spec) where
    the spec holds the generator arguments; ``materialize_problem`` builds it.
    """
    g = _rng(seed)
    t = 0.0
    out = []
    for j in range(n_problems):
        K = int(g.integers(K_range[0], K_range[1] + 1))
        if max_K is not None:
            K = min(K, max_K)
        Nk = g.integers(Nk_range[0], Nk_range[1] + 1, size=K).astype(np.int64)
        if max_Nk is not None:
            Nk = np.minimum(Nk, max_Nk)
        sub_seed = int(g.integers(0, 2**62))
        if rate is not None:
            t += float(g.exponential(1.0 / rate))
        out.append((t, dict(kind="harmonic" if j % 2 == 0 else "double_well", K=K, Nk=Nk,
                            seed=sub_seed)))
    return out


def materialize_problem(spec, materialize=True):
    """Build a stream problem; ``materialize=False`` leaves u to the model (u = None)."""
    if spec["kind"] == "harmonic":
        return harmonic_1d(K=spec["K"], Nk=spec["Nk"], seed=spec["seed"],
                           materialize=materialize)
    K = spec["K"]
    kappa = 50.0 * ((K - 1) / 99.0) ** 2
    return double_well_iid(K, spec["Nk"], kappa, spec["seed"], materialize=materialize)


def config(i, seed=None, scale=1.0):
    """Workloads 0-4 at full size (scale = 1) or with sample counts scaled down."""
    if i == 0:
        return harmonic_1d(K=8, Nk=max(2, int(1000 * scale)), seed=0 if seed is None else seed)
    if i == 1:
        return double_well(K=100, Nk=max(2, int(10000 * scale)), seed=1 if seed is None else seed)
    if i == 2:
        return ladder_2d(K=1000, Nk=max(2, int(2000 * scale)), seed=2 if seed is None else seed)
    if i == 4:
        return muller_brown_grid(G=40, Nk=max(2, int(5000 * scale)),
                                 seed=4 if seed is None else seed)
    raise ValueError("workload 3 is a stream: use serving_stream()")
