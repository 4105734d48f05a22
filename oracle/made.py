"""MADE: masked one-hidden-layer autoencoder (paper Sec. 2.3, MADE layer equations;
architecture MaskedFC1 -> ReLU -> MaskedFC2 -> Sigmoid of Sec. 5.1), in float64.

    g1(s) = max(0, (M1 . W1) s + b1)              hidden activations r   (h)
    g2(s) = sigmoid((M2 . W2) g1(s) + b2)         conditionals p        (n)

with pi(s) = prod_d pi_d(s_d | s_<d) (Sec. 2.3, autoregressive factorisation) and
pi_d(+1 | s_<d) = p_d (reading R2).  Masks follow the MADE degree rule (reading R3).
"""
from __future__ import annotations

import numpy as np


def masks(n: int, degrees) -> tuple[np.ndarray, np.ndarray]:
    """M1 (h x n) and M2 (n x h) as float64 0/1 arrays.

    Unit k with degree m(k) (1-based, in [1, n-1]) receives input site d (1-based) iff
    d <= m(k), and output site d depends on unit k iff d > m(k)."""
    m = np.asarray(degrees, dtype=np.int64)
    if m.min() < 1 or m.max() > n - 1:
        raise ValueError("degrees must lie in [1, n-1]")
    site = np.arange(1, n + 1)
    M1 = (site[None, :] <= m[:, None]).astype(np.float64)
    M2 = (site[:, None] > m[None, :]).astype(np.float64)
    return M1, M2


def log_sigmoid(t) -> np.ndarray:
    """log sigma(t) = min(t, 0) - log1p(exp(-|t|)) (reading R9)."""
    t = np.asarray(t, dtype=np.float64)
    return np.minimum(t, 0.0) - np.log1p(np.exp(-np.abs(t)))


def sigmoid(t) -> np.ndarray:
    t = np.asarray(t, dtype=np.float64)
    e = np.exp(-np.abs(t))
    return np.where(t >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def as_f64(params: dict) -> dict:
    """Parameters widened to float64 (the oracle's working precision)."""
    out = {k: np.asarray(params[k], dtype=np.float64) for k in ("W1", "b1", "W2", "b2")}
    out["degrees"] = np.asarray(params["degrees"])
    return out


def forward(params: dict, S) -> dict:
    """Dense masked forward pass on a batch of spin strings S (B x n, entries +-1).

    Returns A = (M1.W1) S^T + b1 (pre-activations, B x h), R = relu(A),
    Z = (M2.W2) R + b2 (logits, B x n) and logp[b] = sum_d log sigma(s_d z_d)."""
    p = as_f64(params)
    S = np.asarray(S, dtype=np.float64)
    n = S.shape[1]
    M1, M2 = masks(n, p["degrees"])
    A = S @ (M1 * p["W1"]).T + p["b1"]
    R = np.maximum(A, 0.0)
    Z = R @ (M2 * p["W2"]).T + p["b2"]
    logp = log_sigmoid(S * Z).sum(axis=1)
    return {"A": A, "R": R, "Z": Z, "logp": logp}


def logp(params: dict, S) -> np.ndarray:
    return forward(params, S)["logp"]


def conditionals(params: dict, S) -> np.ndarray:
    """p[b, d] = P(s_d = +1 | s_<d) evaluated on the prefixes of the given strings."""
    return sigmoid(forward(params, S)["Z"])
