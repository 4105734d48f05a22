"""Batch estimators of Sec. 2.1 and the gradient of log pi through MADE, in float64.

Population forms (Sec. 2.1): L = E_pi[l], var = E_pi[(l - L)^2] (eq. stochastic_variance),
grad L = 2 E_pi[(l - L) grad log|psi|].  With psi = sqrt(pi) (Sec. 2.3),
2 grad log|psi| = grad log pi.  Batch form (reading R6): with the batch mean as baseline,

    Lhat = mean_b E_b,  var = sum_b (E_b - Lhat)^2 / B,  c_b = (E_b - Lhat) / B,
    g    = sum_b c_b grad log pi(s_b).

For a diagonal Hamiltonian E does not depend on theta, so E[g] = (1 - 1/B) grad L exactly.
"""
from __future__ import annotations

import numpy as np

from . import made


def batch_stats(E, W_tot=None) -> dict:
    """mean, population variance, min, first argmin, the gradient coefficients c_b,
    and (for graphs) best and mean cut values."""
    E = np.asarray(E)
    Ef = E.astype(np.float64)
    B = Ef.shape[0]
    mean = Ef.sum() / B
    var = ((Ef - mean) ** 2).sum() / B
    out = {"mean": mean, "var": var, "min": E.min(), "argmin": int(np.argmin(E)),
           "coef": (Ef - mean) / B}
    if W_tot is not None:
        out["best_cut"] = (W_tot - E.min()) / 2
        out["mean_cut"] = (W_tot - mean) / 2
    return out


def logp_grad(params: dict, S, coef, active=None) -> dict:
    """Gradient of F(theta) = sum_b coef_b log pi(s_b) with respect to W1, b1, W2, b2.

    Chain rule through the MADE forward pass:
        dF/dz_bd  = coef_b s_bd sigma(-s_bd z_bd)           (d/dt log sigma(t) = sigma(-t))
        dF/dW2    = M2 . (G^T R),          dF/db2 = sum_b G
        dF/da_bk  = [a_bk > 0] (G (M2.W2))_bk                (reading R10 at a = 0)
        dF/dW1    = M1 . (Ga^T S),         dF/db1 = sum_b Ga
    Masked entries of dW1/dW2 are exactly zero.

    ``active`` (optional, B x h booleans) replaces the ReLU gate [a_bk > 0] where a caller
    has to take a pre-activation's side from elsewhere: a pre-activation within rounding of
    0 has no well-defined side in finite precision, so a parity test takes the side the
    evaluated path took there (as the sampled spins are teacher-forced) and the oracle's
    own sign everywhere else."""
    p = made.as_f64(params)
    S = np.asarray(S, dtype=np.float64)
    coef = np.asarray(coef, dtype=np.float64)
    n = S.shape[1]
    M1, M2 = made.masks(n, p["degrees"])
    f = made.forward(params, S)
    G = coef[:, None] * S * made.sigmoid(-S * f["Z"])
    dW2 = M2 * (G.T @ f["R"])
    db2 = G.sum(axis=0)
    gate = f["A"] > 0 if active is None else np.asarray(active, dtype=bool)
    Ga = (G @ (M2 * p["W2"])) * gate
    dW1 = M1 * (Ga.T @ S)
    db1 = Ga.sum(axis=0)
    return {"W1": dW1, "b1": db1, "W2": dW2, "b2": db2}


def score_gradient(params: dict, S, E) -> dict:
    """g = sum_b c_b grad log pi(s_b) with c from :func:`batch_stats` (reading R6)."""
    return logp_grad(params, S, batch_stats(E)["coef"])


def finite_difference_grad(params: dict, S, coef, eps: float = 1e-6,
                           names=("W1", "b1", "W2", "b2")) -> dict:
    """Central differences of F(theta) = sum_b coef_b log pi(s_b), one parameter at a
    time, in float64 (masked weights included: their derivative must be 0)."""
    S = np.asarray(S, dtype=np.float64)
    coef = np.asarray(coef, dtype=np.float64)
    base = made.as_f64(params)

    def F(pp):
        return float(coef @ made.logp(pp, S))

    out = {}
    for name in names:
        arr = base[name]
        g = np.zeros_like(arr)
        it = np.nditer(arr, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            plus = dict(base)
            minus = dict(base)
            a_p = arr.copy()
            a_m = arr.copy()
            a_p[idx] += eps
            a_m[idx] -= eps
            plus[name] = a_p
            minus[name] = a_m
            g[idx] = (F(plus) - F(minus)) / (2 * eps)
        out[name] = g
    return out
