"""Brute force over all 2^n spin strings (small n only), float64.

Gives the exact normalisation sum_s pi(s) (Sec. 2.3: the autoregressive product is
normalised), the exact objective L = E_pi[E] and its gradient
grad L = E_pi[(E - L) grad log pi] (Sec. 2.1), the variational bound L >= lambda_min
(Sec. 2.1), and the exact Max-Cut optimum.
"""
from __future__ import annotations

import numpy as np

from . import made
from .estimator import logp_grad


def all_strings(n: int) -> np.ndarray:
    """All 2^n strings in {-1,+1}^n (int8), string index x -> s_i = 1 - 2 * bit_i(x)
    with site 0 the most significant bit (the paper's x = 2^{n-1} x_1 ... 2^0 x_n)."""
    if n > 24:
        raise ValueError("n too large for enumeration")
    x = np.arange(2 ** n, dtype=np.int64)
    bits = (x[:, None] >> np.arange(n - 1, -1, -1, dtype=np.int64)[None, :]) & 1
    return (1 - 2 * bits).astype(np.int8)


def log_probs(params: dict, n: int, chunk: int = 1 << 16) -> np.ndarray:
    S = all_strings(n)
    out = np.empty(S.shape[0], dtype=np.float64)
    for i in range(0, S.shape[0], chunk):
        out[i:i + chunk] = made.logp(params, S[i:i + chunk])
    return out


def exact_objective(params: dict, energies) -> dict:
    """pi over all strings, L, var and grad L for energies indexed like all_strings."""
    n = int(round(np.log2(len(energies))))
    lp = log_probs(params, n)
    pi = np.exp(lp)
    E = np.asarray(energies, dtype=np.float64)
    L = float(pi @ E)
    var = float(pi @ (E - L) ** 2)
    grad = logp_grad(params, all_strings(n), pi * (E - L))
    return {"pi": pi, "L": L, "var": var, "grad": grad, "norm": float(pi.sum())}


def max_cut_brute(n: int, energies, W_tot) -> tuple:
    """(best cut, minimum energy) over all strings."""
    E = np.asarray(energies)
    Emin = E.min()
    return (W_tot - Emin) / 2, Emin
