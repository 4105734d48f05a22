"""float32 -> bfloat16 rounding, round-to-nearest-even, written from the IEEE-754 binary32
layout: bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits.

The paper fixes no precision; the GPU kernels may run on BF16 weights (reading: the oracle
evaluates the model on the BF16-rounded weights, widened back to float64, so that parity
isolates arithmetic error from quantisation).  Pinned against torch's CPU cast.
"""
from __future__ import annotations

import numpy as np


def round_to_bf16(x) -> np.ndarray:
    """Return float32 values that are exactly representable in bfloat16 (RNE)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    rounded = (bits + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = (rounded & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    nan = np.isnan(x)
    if nan.any():
        out = out.copy()
        out[nan] = np.nan
    return out


def bf16_bits(x) -> np.ndarray:
    """The 16-bit patterns of :func:`round_to_bf16` (uint16)."""
    r = round_to_bf16(x)
    return (r.view(np.uint32) >> np.uint32(16)).astype(np.uint16)
