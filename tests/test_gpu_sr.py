"""SR Gram (vqmc_sr_gram) against the oracle's explicit score matrix: K = O O^T over every
unmasked parameter (Sec. 2.1 Fisher information; SR of Sec. 5.1, reading R19).

Tolerance: each entry within rtol * sqrt(K_bb K_b'b') of the FP64 value (the
Cauchy-Schwarz bound on |K_bb'|).  FP32: rtol 2e-4 -- the factors G, R, D are FP32
(relative error ~1e-6) and every entry accumulates 3 (n + h) products in FP32.  BF16: rtol
2e-2 -- the factors are stored in BF16 (relative rounding 2^-9 each)."""
import numpy as np
import pytest
import torch

from oracle import sr as osr
from paper_2106_13308_amd import inputs

from gpu_util import DEV, build_made, oracle_params

pytestmark = pytest.mark.gpu

RTOL = {"f32": 2e-4, "bf16": 2e-2}


@pytest.mark.parametrize("wd", ["f32", "bf16"])
@pytest.mark.parametrize("n,h,B", [(20, 40, 64), (67, 33, 100), (130, 70, 200), (300, 200, 70), (9, 3, 1), (64, 64, 130)])
def test_sr_gram_matches_oracle(wd, n, h, B):
    from paper_2106_13308_amd import binding as Bd
    wdt = Bd.F32 if wd == "f32" else Bd.BF16
    print(f"[sr-gram] wd={wd} n={n} h={h} B={B}", flush=True)
    p = inputs.made_init(n, h, 61)
    S = inputs.random_spins(B, n, 62)
    made = build_made(p, wdt)
    Sd = torch.zeros((B, Bd.ld(n)), dtype=torch.int8, device=DEV)
    Sd[:, :n] = torch.from_numpy(S).to(DEV)
    K = Bd.sr_gram(made, Sd, B).double().cpu().numpy()
    torch.cuda.synchronize()
    Kref = osr.gram(oracle_params(p, wdt), S)
    scale = np.sqrt(np.outer(np.diag(Kref), np.diag(Kref)))
    err = np.abs(K - Kref) / np.maximum(scale, 1e-30)
    assert np.isfinite(K).all()
    assert np.array_equal(K, K.T)                            # mirrored, not recomputed
    assert err.max() <= RTOL[wd], f"max normalised error {err.max():.3g}"


def test_sr_gram_two_calls_and_tile_edges():
    """A second call with a smaller batch overwrites only its own B x B block; the entries
    next to the diagonal tiles (b, b' in different 64-sample tiles) match too."""
    from paper_2106_13308_amd import binding as Bd
    n, h = 90, 70
    p = inputs.made_init(n, h, 71)
    made = build_made(p, Bd.F32)
    for B in (150, 65):
        S = inputs.random_spins(B, n, 72 + B)
        Sd = torch.zeros((B, Bd.ld(n)), dtype=torch.int8, device=DEV)
        Sd[:, :n] = torch.from_numpy(S).to(DEV)
        K = Bd.sr_gram(made, Sd, B).double().cpu().numpy()
        Kref = osr.gram(oracle_params(p, Bd.F32), S)
        scale = np.sqrt(np.outer(np.diag(Kref), np.diag(Kref)))
        assert (np.abs(K - Kref) / scale).max() <= RTOL["f32"]
        assert abs(K[63, 64] - Kref[63, 64]) <= RTOL["f32"] * scale[63, 64]


def test_sr_gram_full_size_sampled_entries():
    """At n = 10^4, h = 1000, B = 2048 (BF16 factors, the launch the bench times) the oracle
    forms the score rows of six samples spread over the batch (different 64-sample tiles and
    work items) and every entry of K among them is checked."""
    from paper_2106_13308_amd import binding as Bd
    n, h, B = 10000, 1000, 2048
    w = inputs.WORKLOADS["maxcut10k"]
    assert (w.n, w.h, w.B) == (n, h, B)
    p = inputs.made_init(n, h, 1)
    S = inputs.random_spins(B, n, 81)
    made = build_made(p, Bd.BF16)
    Sd = torch.zeros((B, Bd.ld(n)), dtype=torch.int8, device=DEV)
    Sd[:, :n] = torch.from_numpy(S).to(DEV)
    print(f"[sr-gram] full size n={n} h={h} B={B}", flush=True)
    K = Bd.sr_gram(made, Sd, B)
    torch.cuda.synchronize()
    idx = np.array([0, 63, 64, 1000, 2046, 2047])
    Ks = K[idx][:, idx].double().cpu().numpy()
    O = osr.score_matrix(oracle_params(p, Bd.BF16), S[idx])
    Kref = O @ O.T
    scale = np.sqrt(np.outer(np.diag(Kref), np.diag(Kref)))
    err = np.abs(Ks - Kref) / scale
    assert err.max() <= RTOL["bf16"], f"max normalised error {err.max():.3g}"


@pytest.mark.parametrize("wd", ["f32", "bf16"])
@pytest.mark.parametrize("n,h,B", [(67, 33, 100), (130, 70, 200), (20, 40, 64)])
def test_sr_gram_sampled_matches_oracle(wd, n, h, B):
    """vqmc_sr_gram_sampled on the spins vqmc_sample_fwd drew, from its Zs and Rt, against the
    oracle's Gram of the same spins."""
    from paper_2106_13308_amd import binding as Bd
    wdt = Bd.F32 if wd == "f32" else Bd.BF16
    print(f"[sr-gram-sampled] wd={wd} n={n} h={h} B={B}", flush=True)
    p = inputs.made_init(n, h, 91)
    made = build_made(p, wdt)
    S, _, Zs, Rt = Bd.sample_fwd(made, B, 5, 3)
    K = Bd.sr_gram_sampled(made, S, Zs, Rt, B).double().cpu().numpy()
    torch.cuda.synchronize()
    Snp = S[:, :n].cpu().numpy()
    Kref = osr.gram(oracle_params(p, wdt), Snp)
    scale = np.sqrt(np.outer(np.diag(Kref), np.diag(Kref)))
    err = np.abs(K - Kref) / np.maximum(scale, 1e-30)
    assert np.array_equal(K, K.T)
    assert err.max() <= RTOL[wd], f"max normalised error {err.max():.3g}"
