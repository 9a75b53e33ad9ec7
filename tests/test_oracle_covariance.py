"""Pins of the oracle's asymptotic covariance of f (no GPU).

The oracle evaluates Theta = W^T (I - W diag(N) W^T)^+ W through a thin SVD.
It is pinned here by what does not depend on that evaluation:

* K = 2: the covariance of f_1 - f_0 is the asymptotic variance of Bennett's
  acceptance ratio (BAR) estimate, a closed form in the Fermi function of the
  energy differences at the solution (Shirts, Bair, Hooker, Pande, Phys. Rev.
  Lett. 91, 140601 (2003));
* tiny N: the same Theta with the N x N pseudo-inverse formed directly;
* an unsampled copy of a sampled state has its free energy exactly, so the
  variance of their difference is zero and their covariance rows agree;
* gauge: Cov(f_0, .) = 0 and the result does not change under u_k + c_k;
* 16 seeded repetitions of harmonic wells (one state unsampled), whose free
  energies are known in closed form: the standardised errors have mean
  square near 1 (a missing -1/N_k term inflates the variance 2-8 fold here).
"""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module", autouse=True)
def built():
    oracle.build()


def test_two_states_is_bar_variance():
    for seed, nk in ((2, [300, 500]), (5, [50, 900]), (8, [400, 400])):
        p = synth.harmonic_1d(K=2, Nk=nk, seed=seed)
        f, _ = oracle.solve_mbar(p["u"], p["Nk"])
        C = oracle.covariance(p["u"], p["Nk"], f)
        N0, N1 = p["Nk"]
        N = N0 + N1
        # the work W = u_1 - u_0 on all N pooled samples, M = ln(N_0 / N_1)
        # (state 0 the forward side), and the estimate dF = f_1 - f_0
        x = np.log(N0 / N1) + (p["u"][1] - p["u"][0]) - (f[1] - f[0])
        var = (1.0 / np.mean(1.0 / (2.0 + 2.0 * np.cosh(x))) - N / N0 - N / N1) / N
        assert abs(C[1, 1] / var - 1.0) < 1e-10
        assert abs(C[0, 0]) + abs(C[0, 1]) < 1e-14 * C[1, 1]


def test_tiny_n_direct_pseudo_inverse():
    p = synth.harmonic_1d(K=5, Nk=[12, 0, 9, 15, 7], seed=3)
    f, _ = oracle.solve_mbar(p["u"], p["Nk"])
    W = oracle.weights(p["u"], p["Nk"], f)
    N = W.shape[0]
    theta = W.T @ np.linalg.pinv(np.eye(N) - W @ np.diag(p["Nk"].astype(float)) @ W.T,
                                 rcond=1e-9) @ W
    ref = theta - theta[:, :1] - theta[:1, :] + theta[0, 0]
    C = oracle.covariance(p["u"], p["Nk"], f)
    assert np.max(np.abs(C - ref)) < 1e-9 * np.max(np.abs(ref))


def test_unsampled_copy_and_gauge():
    p = synth.harmonic_1d(K=4, Nk=[200, 300, 250, 280], seed=4)
    u = np.vstack([p["u"], p["u"][2:3]])  # state 4 = state 2, never sampled
    Nk = np.append(p["Nk"], 0)
    f, _ = oracle.solve_mbar(u, Nk)
    C = oracle.covariance(u, Nk, f)
    scale = np.max(np.abs(C))
    assert abs(C[4, 4] + C[2, 2] - 2 * C[2, 4]) < 1e-10 * scale
    assert np.max(np.abs(C[4] - C[2])) < 1e-10 * scale
    assert np.max(np.abs(C[0])) + np.max(np.abs(C[:, 0])) < 1e-14 * scale
    assert np.max(np.abs(C - C.T)) < 1e-13 * scale
    assert np.all(np.linalg.eigvalsh(C[1:, 1:]) > -1e-12 * scale)
    shift = np.array([3.0, -1.0, 0.5, 7.0, 2.0])
    f2, _ = oracle.solve_mbar(u + shift[:, None], Nk)
    C2 = oracle.covariance(u + shift[:, None], Nk, f2)
    assert np.max(np.abs(C2 - C)) < 1e-8 * scale


def test_seeded_repetitions_match_the_predicted_variance():
    kappa = np.array([2.0, 1.5, 3.0, 2.5])
    x0 = np.array([-0.8, -0.2, 0.3, 0.9])
    Nk = np.array([300, 400, 0, 350])
    f_true = 0.5 * np.log(kappa / kappa[0])  # f_k = -ln sqrt(2 pi / kappa_k), gauge f_0 = 0
    z2 = []
    for seed in range(16):
        g = np.random.Generator(np.random.PCG64(1000 + seed))
        x = np.concatenate([g.normal(x0[k], 1 / np.sqrt(kappa[k]), Nk[k]) for k in range(4)])
        u = 0.5 * kappa[:, None] * (x[None, :] - x0[:, None]) ** 2
        f, _ = oracle.solve_mbar(u, Nk)
        C = oracle.covariance(u, Nk, f)
        z2.append((f[1:] - f_true[1:]) ** 2 / np.diag(C)[1:])
    m = float(np.mean(z2))
    assert 0.45 < m < 1.8, m
