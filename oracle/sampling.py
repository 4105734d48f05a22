"""Autoregressive sampling, Algorithm 1 of the paper ("Autoregressive Sampling"): for each
site i in order, compute p(x_i | x_<i) with a forward pass, draw x_i from it, write it
into the state.  The uniforms u are inputs (drawn by :mod:`oracle.philox`), and
s_d = +1 iff u[b, d] < p_d (reading R8).

Two independent float64 implementations:

* :func:`sample_literal` - exactly Algorithm 1: a full dense masked forward pass of the
  whole batch for every site (n passes, O(n^2 h) per sample).  For small n.
* :func:`sample_plain`   - the same draws, but each hidden pre-activation a_k is
  computed fresh from its definition b1_k + sum_{d <= m(k)} W1[k, d] s_d at the moment its
  last input site m(k) has been drawn, and each logit z_d is a fresh dot product over
  the units it depends on.  No state is carried between sites other than the drawn
  spins and the finished activations; O(n h) per sample, usable at n = 10^4.

Both return (S, logp): int8 spins (B x n) and log pi(S) (float64, B).
"""
from __future__ import annotations

import numpy as np

from . import made


def sample_literal(params: dict, U, x0=None):
    """Algorithm 1 with a full forward pass per site.

    x0 is the random initial state of Algorithm 1 (B x n, +-1); the masks make its
    value irrelevant, which the tests check by passing different x0."""
    U = np.asarray(U, dtype=np.float64)
    B, n = U.shape
    X = np.ones((B, n), dtype=np.float64) if x0 is None else np.asarray(x0, np.float64).copy()
    for i in range(n):
        p = made.conditionals(params, X)[:, i]       # forward pass on x^{i-1}
        X[:, i] = np.where(U[:, i] < p, 1.0, -1.0)   # sample y_i, write x^i
    lp = made.logp(params, X)
    return X.astype(np.int8), lp


def sample_plain(params: dict, U):
    """Algorithm 1 evaluated unit by unit from the definitions (see module docstring)."""
    p = made.as_f64(params)
    U = np.asarray(U, dtype=np.float64)
    B, n = U.shape
    W1, b1, W2, b2 = p["W1"], p["b1"], p["W2"], p["b2"]
    m = np.asarray(p["degrees"], dtype=np.int64)
    h = m.shape[0]
    S = np.zeros((B, n), dtype=np.float64)
    R = np.zeros((B, h), dtype=np.float64)          # finished activations relu(a_k)
    lp = np.zeros(B, dtype=np.float64)
    for d in range(1, n + 1):                        # 1-based site index
        feeds = np.nonzero(m < d)[0]                 # units with m(k) < d feed output d
        z = b2[d - 1] + R[:, feeds] @ W2[d - 1, feeds]
        pd = made.sigmoid(z)
        s = np.where(U[:, d - 1] < pd, 1.0, -1.0)
        S[:, d - 1] = s
        lp += made.log_sigmoid(s * z)
        for k in np.nonzero(m == d)[0]:              # units whose last input is site d
            a = b1[k] + S[:, :d] @ W1[k, :d]
            R[:, k] = np.maximum(a, 0.0)
    return S.astype(np.int8), lp


def teacher_forced_check(params: dict, S, U, tau: float):
    """Check sampled spins against the oracle's conditionals on their own prefixes.

    For every (b, d) with |u - p_ref| > tau the spin must equal +1 iff u < p_ref, where
    p_ref is the oracle's conditional evaluated on S's prefix.  Returns
    (n_mismatch, n_ambiguous, p_ref)."""
    S = np.asarray(S)
    U = np.asarray(U, dtype=np.float64)
    pref = made.conditionals(params, S)
    want = np.where(U < pref, 1, -1)
    decided = np.abs(U - pref) > tau
    mismatch = int(np.count_nonzero((want != S) & decided))
    return mismatch, int(np.count_nonzero(~decided)), pref
