"""Stochastic reconfiguration (natural gradient) quantities, in float64 (Sec. 2.1: the
Fisher information I(theta) = E_pi[grad log pi (x) grad log pi], used with a ridge
lambda (Sec. 5.1)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Batch forms (reading R19): with the per-sample scores O[b] = grad log pi(s_b) as the
rows of O (B x d, over every unmasked parameter: W1 and W2 inside their masks, b1, b2),

    I_hat = O^T O / B                                   (the expectation as printed: uncentred)
    K     = O O^T                                       (B x B sample-space Gram)
    x     = (I_hat + lambda I_d)^{-1} g                 (the SR direction for a gradient g)
          = (g - O^T (lambda B I_B + K)^{-1} O g) / lambda     (Woodbury identity)

When g is the batch gradient itself, g = O^T c with the coefficients c_b of Sec. 2.1
(reading R6), the push-through identity (O^T O / B + lambda I) O^T = O^T (K / B + lambda I)
gives the direction without any d-dimensional solve or division by lambda:

    x = O^T y,   (K + lambda B I_B) y = B c.

``sr_direction`` solves the d x d system as written; ``sr_direction_woodbury`` goes
through K for any g; ``sr_direction_coef`` takes c and uses the push-through form.  Nothing here is blocked or fused: O is formed explicitly, one sample at a
time, from :func:`oracle.estimator.logp_grad`.
"""
from __future__ import annotations

import numpy as np

from . import estimator, made


def flatten(params: dict, grads: dict) -> np.ndarray:
    """The unmasked entries of (W1, b1, W2, b2) as one vector: W1 inside M1 (row-major),
    b1, W2 inside M2 (row-major), b2."""
    n = np.asarray(grads["b2"]).shape[-1]
    M1, M2 = made.masks(n, params["degrees"])
    return np.concatenate([np.asarray(grads["W1"])[M1 > 0], np.asarray(grads["b1"]),
                           np.asarray(grads["W2"])[M2 > 0], np.asarray(grads["b2"])])


def score_matrix(params: dict, S) -> np.ndarray:
    """O (B x d): row b is grad log pi(s_b) over the unmasked parameters."""
    S = np.asarray(S)
    rows = [flatten(params, estimator.logp_grad(params, S[b:b + 1], np.ones(1))) for b in range(S.shape[0])]
    return np.stack(rows)


def fisher(params: dict, S) -> np.ndarray:
    """I_hat = O^T O / B (d x d)."""
    O = score_matrix(params, S)
    return O.T @ O / O.shape[0]


def gram(params: dict, S) -> np.ndarray:
    """K = O O^T (B x B): K[b, b'] = <grad log pi(s_b), grad log pi(s_b')>."""
    O = score_matrix(params, S)
    return O @ O.T


def sr_direction(params: dict, S, g, lam: float) -> np.ndarray:
    """x solving (O^T O / B + lambda I) x = g, as a d x d linear system."""
    O = score_matrix(params, S)
    d = O.shape[1]
    return np.linalg.solve(O.T @ O / O.shape[0] + lam * np.eye(d), np.asarray(g, np.float64))


def sr_direction_woodbury(params: dict, S, g, lam: float) -> np.ndarray:
    """The same x through the B x B Gram: x = (g - O^T (lambda B I + K)^{-1} O g) / lambda."""
    O = score_matrix(params, S)
    B = O.shape[0]
    g = np.asarray(g, np.float64)
    y = np.linalg.solve(lam * B * np.eye(B) + O @ O.T, O @ g)
    return (g - O.T @ y) / lam


def sr_direction_coef(params: dict, S, coef, lam: float) -> np.ndarray:
    """x for g = O^T c (the batch gradient of Sec. 2.1 with coefficients c): y solves
    (K + lambda B I) y = B c and x = O^T y."""
    O = score_matrix(params, S)
    B = O.shape[0]
    y = np.linalg.solve(O @ O.T + lam * B * np.eye(B), B * np.asarray(coef, np.float64))
    return O.T @ y
