"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11, Sec. 3-4) and the uniform variates the sampler
draws from it.

The paper only says samples are drawn from the conditionals (Algorithm 1, "Sample y_i")
by transforming i.i.d. variates of a simple distribution (Sec. 4).  Reading R8: each
(sample b, site d) pair gets one uniform u[b, d] in [0, 1) with 24 random bits,

    block   = Philox4x32-10(counter = (d // 4, b, step, tag), key = (seed_lo, seed_hi))
    u[b, d] = (block[d % 4] >> 8) * 2**-24

so u is exactly representable in float32 and float64.

Pinned by the published known-answer vectors of the Random123 distribution
(``tests/golden/philox4x32_10_kat.txt``).
"""
from __future__ import annotations

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)   # multiplier applied to counter word 0
_M1 = np.uint64(0xCD9E8D57)   # multiplier applied to counter word 2
_W0 = np.uint64(0x9E3779B9)   # Weyl key increment, word 0 (golden ratio)
_W1 = np.uint64(0xBB67AE85)   # Weyl key increment, word 1 (sqrt(3) - 1)
_S32 = np.uint64(32)


def philox4x32_10(counter, key) -> np.ndarray:
    """Philox4x32 with 10 rounds.

    counter: (..., 4) uint32-valued array; key: (..., 2) uint32-valued array (broadcast).
    Returns the (..., 4) uint32 output block.

    One round maps (c0, c1, c2, c3) with key (k0, k1) to
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
    the key is advanced by the Weyl constants between rounds.
    """
    counter = np.asarray(counter, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (counter[..., i] for i in range(4))
    k0, k1 = key[..., 0], key[..., 1]
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0                       # < 2**64: exact in uint64
        p1 = _M1 * c2
        c0, c1, c2, c3 = ((p1 >> _S32) ^ c1 ^ k0, p1 & _MASK,
                          (p0 >> _S32) ^ c3 ^ k1, p0 & _MASK)
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


TAG_TRAIN = 0
TAG_EVAL = 1


def uniforms(seed: int, step: int, sample_ids, n: int, tag: int = TAG_TRAIN) -> np.ndarray:
    """u[b, d] for the given global sample indices and sites 0..n-1 (float64, 24-bit)."""
    sample_ids = np.asarray(sample_ids, dtype=np.uint64)
    nblk = (n + 3) // 4
    B = sample_ids.shape[0]
    ctr = np.zeros((B, nblk, 4), dtype=np.uint64)
    ctr[..., 0] = np.arange(nblk, dtype=np.uint64)[None, :]
    ctr[..., 1] = (sample_ids & _MASK)[:, None]
    ctr[..., 2] = np.uint64(step) & _MASK
    ctr[..., 3] = np.uint64(tag) & _MASK
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    words = philox4x32_10(ctr, key).reshape(B, nblk * 4)[:, :n]
    return (words >> np.uint32(8)).astype(np.float64) * 2.0 ** -24
