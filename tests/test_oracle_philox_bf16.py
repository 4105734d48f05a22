"""Pins for the oracle's Philox4x32-10 and its BF16 rounding (CPU only)."""
import os

import numpy as np
import pytest
import torch

from oracle import philox, bf16

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answer_vectors():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = philox.philox4x32_10(np.array(ctr, np.uint64), np.array(key, np.uint64))
        assert [int(x) for x in got] == want


def test_philox_vectorised_matches_scalar_calls():
    rng = np.random.default_rng(5)
    ctr = rng.integers(0, 2 ** 32, size=(7, 4), dtype=np.uint64)
    key = rng.integers(0, 2 ** 32, size=(7, 2), dtype=np.uint64)
    many = philox.philox4x32_10(ctr, key)
    for i in range(7):
        assert np.array_equal(many[i], philox.philox4x32_10(ctr[i], key[i]))


def test_uniforms_layout_and_range():
    u = philox.uniforms(seed=2, step=3, sample_ids=np.arange(5), n=10)
    assert u.shape == (5, 10)
    assert (u >= 0).all() and (u < 1).all()
    # 24-bit dyadic: exactly representable in float32
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    assert np.array_equal((u * 2 ** 24), np.floor(u * 2 ** 24))
    # site d of sample b is word d % 4 of the block with counter (d // 4, b, step, tag)
    blk = philox.philox4x32_10(np.array([2, 4, 3, 0], np.uint64), np.array([2, 0], np.uint64))
    assert u[4, 9] == (int(blk[1]) >> 8) / 2 ** 24
    # a different step / tag / seed gives a different stream
    assert not np.array_equal(u, philox.uniforms(2, 4, np.arange(5), 10))
    assert not np.array_equal(u, philox.uniforms(2, 3, np.arange(5), 10, tag=1))
    assert not np.array_equal(u, philox.uniforms(3, 3, np.arange(5), 10))
    # the sample index is global: a shard reproduces the rows of the full batch
    assert np.array_equal(philox.uniforms(2, 3, np.arange(3, 5), 10), u[3:5])


def test_uniforms_chi2_and_serial_correlation():
    u = philox.uniforms(seed=11, step=0, sample_ids=np.arange(4096), n=256).ravel()
    counts = np.bincount((u * 256).astype(np.int64), minlength=256)
    exp = u.size / 256
    chi2 = ((counts - exp) ** 2 / exp).sum()
    # 255 dof: mean 255, sd ~22.6; 6 sd band
    assert 120 < chi2 < 400
    x = u - 0.5
    r1 = (x[:-1] @ x[1:]) / (x @ x)
    assert abs(r1) < 6 / np.sqrt(u.size)
    assert abs(u.mean() - 0.5) < 6 * np.sqrt(1 / 12 / u.size)


def test_bf16_round_matches_torch_cpu_cast():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(100000).astype(np.float32),
        rng.uniform(-1e-3, 1e-3, 1000).astype(np.float32),
        np.array([0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, 3.4e38, 1e-40, -1e-42], np.float32),
        # exact ties: low 16 bits == 0x8000, both parities of bit 16
        np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x00018000], np.uint32).view(np.float32),
    ])
    mine = bf16.round_to_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mine.view(np.uint32), ref.view(np.uint32))
    assert np.array_equal(bf16.bf16_bits(x), torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16))
    assert np.isnan(bf16.round_to_bf16(np.array([np.nan], np.float32))[0])
