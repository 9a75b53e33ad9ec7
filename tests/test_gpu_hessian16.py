"""The FP16-core Newton Hessian (K > 256) against the FP64 oracle and, where the
oracle cannot hold u, against the FP64 matrix-core Hessian of the same data.

H_ij = delta_ij S_i - sum_n P_in P_jn (Section 2, derivative-based finisher)
with P rounded to FP16 in a sample-tiled copy: each product carries at most
about 2^-10 relative error and the sums are of positive terms, so every
element lies within 1e-3 of the largest |H_ij|. The copy holds at most 4 GiB
(2^31 / K samples); the full-size cases cross that cap, so the product adds
the super-chunks into the same partial blocks.
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


def windows_1d(K, N, seed, unsampled=()):
    """1-D harmonic windows: centres, force constants, counts and the samples."""
    g = np.random.default_rng(seed)
    Nk = np.zeros(K, dtype=np.int64)
    sampled = [k for k in range(K) if k not in unsampled]
    Nk[sampled] = N // len(sampled)
    Nk[sampled[0]] += N - Nk.sum()
    c = np.sort(g.uniform(-3, 3, K))
    kap = g.uniform(20, 80, K)
    owner = np.repeat(np.arange(K), Nk)
    x = g.normal(c[owner], 1 / np.sqrt(kap[owner]))
    return Nk, x, c, kap


@pytest.mark.parametrize("K,N,dtype", [(257, 1001, "f64"), (300, 4099, "f32"),
                                       (700, 2003, "f64"), (520, 777, "f32")])
def test_fp16_hessian_matches_oracle(bm, K, N, dtype):
    import torch
    say(f"fp16 hessian K={K} N={N} {dtype}")
    Nk, x, c, kap = windows_1d(K, N, seed=K + N, unsampled=(1, K // 2))
    u = 0.5 * kap[:, None] * (x[None, :] - c[:, None]) ** 2
    if dtype == "f32":
        u = u.astype(np.float32).astype(np.float64)
    f = np.concatenate([[0.0], np.random.default_rng(K).normal(0, 0.3, K - 1)])
    H_ref = oracle.hessian(u, Nk, f)
    ud = torch.as_tensor(u.astype(np.float32) if dtype == "f32" else u).cuda()
    _, lD, S, _ = bm.sweep(ud, Nk, f)
    H = bm.hessian(ud, Nk, f, lD, S, fp16=True).cpu().numpy()
    scale = np.abs(H_ref).max()
    assert np.max(np.abs(H - H_ref)) < 1e-3 * scale
    assert np.array_equal(H, H.T)
    for k in (1, K // 2):
        assert not H[k].any() and not H[:, k].any()


def test_fp16_hessian_rejects_small_k(bm):
    import torch
    Nk, x, c, kap = windows_1d(256, 1000, seed=3)
    u = torch.as_tensor(0.5 * kap[:, None] * (x[None, :] - c[:, None]) ** 2).cuda()
    f = np.zeros(256)
    _, lD, S, _ = bm.sweep(u, Nk, f)
    with pytest.raises(bm.BumbarError):
        bm.hessian(u, Nk, f, lD, S, fp16=True)


def test_fp16_hessian_super_chunks_stored(bm):
    # K = 300, N = 9e6 FP32 u (10.8 GB): 2^31 / 300 = 7158272 samples per
    # super-chunk, so the second adds 1.84e6 samples into the partial blocks
    import torch
    K, N = 300, 9_000_000
    assert N > (2 ** 31 // K) // 32 * 32
    say(f"fp16 hessian super-chunks K={K} N={N}")
    Nk, x, c, kap = windows_1d(K, N, seed=11)
    coef = np.stack([np.zeros(K), kap, c], axis=1)
    u = bm.model_energies(x[:, None], coef, bm.MODEL_HARMONIC, K, dtype=torch.float32)
    f = np.zeros(K)
    _, lD, S, _ = bm.sweep(u, Nk, f)
    H64 = bm.hessian(u, Nk, f, lD, S).cpu().numpy()
    H16 = bm.hessian(u, Nk, f, lD, S, fp16=True).cpu().numpy()
    del u
    torch.cuda.empty_cache()
    scale = np.abs(H64).max()
    err = np.max(np.abs(H16 - H64))
    say(f"  max |H16 - H64| / scale = {err / scale:.2e}")
    assert err < 1e-3 * scale


def test_fp16_model_hessian_grid_full_size(bm):
    # the 40 x 40 Muller-Brown umbrella grid, K = 1600, N = 8e6: the FP32
    # model's P in 6 super-chunks against the FP64 model Hessian
    import torch
    p = synth.muller_brown_grid(G=40, Nk=5000, seed=4, materialize=False)
    K = len(p["Nk"])
    say(f"fp16 model hessian K={K} N={int(p['Nk'].sum())}")
    f = np.zeros(K)
    _, lD, S, _ = bm.sweep_model(p["xi"], p["coef"], p["model_type"], p["Nk"], f)
    H64 = bm.hessian_model(p["xi"], p["coef"], p["model_type"], p["Nk"], f, lD, S).cpu().numpy()
    H16 = bm.hessian_model(p["xi"], p["coef"], p["model_type"], p["Nk"], f, lD, S,
                           precision=bm.PREC_MIXED).cpu().numpy()
    torch.cuda.empty_cache()
    scale = np.abs(H64).max()
    err = np.max(np.abs(H16 - H64))
    say(f"  max |H16 - H64| / scale = {err / scale:.2e}")
    assert err < 1e-3 * scale
    assert np.array_equal(H16, H16.T)
