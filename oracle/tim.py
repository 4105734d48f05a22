"""Local energy of the transverse-field Ising model (TIM), off-diagonal part included, in
float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

eq. (hamiltonian): H = -sum_i (alpha_i X_i + beta_i Z_i) - sum_{i<j} beta_ij Z_i Z_j, with X_i,
Z_i the Pauli matrices acting on site i.  In the computational basis |x>, x in {0,1}^n
(site 1 the most significant bit, as in the binary index of eq. (e:tim)), Z_i |x> = s_i |x>
with s_i = 1 - 2 x_i (reading R1) and X_i flips bit i, so (eq. (e:tim)):

    H_xx          = -sum_i beta_i s_i - sum_{i<j} beta_ij s_i s_j          (reading R20: i < j)
    H_{x, x^(i)}  = -alpha_i            (x^(i): x with bit i flipped), every other entry 0.

The local energy of Sec. 2.1, l(x) = (H psi)(x) / psi(x), with psi = sqrt(pi) (the
non-negative trial state of Sec. 2.3: alpha_i >= 0 makes the ground state non-negative):

    l(x) = H_xx - sum_i alpha_i exp((log pi(x^(i)) - log pi(x)) / 2).

``flip_logratio`` evaluates log pi(x^(i)) - log pi(x) from its definition, one full forward
pass of the flipped strings per site; ``hamiltonian_dense`` builds H itself from Kronecker
products (small n), against which the tests pin the entries and the local energy.
"""
from __future__ import annotations

import numpy as np

from . import made


def diag_energy(beta_i, beta_ij, S) -> np.ndarray:
    """H_xx = -sum_i beta_i s_i - sum_{i<j} beta_ij s_i s_j (strict upper triangle of beta_ij)."""
    S = np.asarray(S, dtype=np.float64)
    b1 = np.asarray(beta_i, dtype=np.float64)
    Bu = np.triu(np.asarray(beta_ij, dtype=np.float64), 1)
    return -(S @ b1) - np.einsum("bi,ij,bj->b", S, Bu, S)


def flip_logratio(params: dict, S, sites=None) -> np.ndarray:
    """D[b, j] = log pi(s_b with site i_j negated) - log pi(s_b), i_j = sites[j] (default all
    sites, 0-based), by re-evaluating log pi on the flipped strings."""
    S = np.asarray(S)
    n = S.shape[1]
    sites = np.arange(n) if sites is None else np.asarray(sites)
    base = made.logp(params, S)
    out = np.empty((S.shape[0], sites.shape[0]), dtype=np.float64)
    for j, i in enumerate(sites):
        F = S.copy()
        F[:, i] = -F[:, i]
        out[:, j] = made.logp(params, F) - base
    return out


def local_energy(params: dict, S, alpha, beta_i, beta_ij) -> np.ndarray:
    """l(x) for every string of S: H_xx - sum_i alpha_i exp(D_i / 2)."""
    D = flip_logratio(params, S)
    off = np.exp(0.5 * D) @ np.asarray(alpha, dtype=np.float64)
    return diag_energy(beta_i, beta_ij, S) - off


def hamiltonian_dense(alpha, beta_i, beta_ij) -> np.ndarray:
    """H of eq. (hamiltonian) as a 2^n x 2^n matrix, built from its definition: Kronecker
    products of I, X, Z with site 1 the leftmost factor (the most significant bit)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    b1 = np.asarray(beta_i, dtype=np.float64)
    b2 = np.asarray(beta_ij, dtype=np.float64)
    n = alpha.shape[0]
    if n > 12:
        raise ValueError("n too large for a dense Hamiltonian")
    I2 = np.eye(2)
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    Z = np.array([[1.0, 0.0], [0.0, -1.0]])

    def op(factors: dict) -> np.ndarray:
        M = np.ones((1, 1))
        for i in range(n):
            M = np.kron(M, factors.get(i, I2))
        return M

    H = np.zeros((2 ** n, 2 ** n))
    for i in range(n):
        H -= alpha[i] * op({i: X}) + b1[i] * op({i: Z})
        for j in range(i + 1, n):
            H -= b2[i, j] * op({i: Z, j: Z})
    return H
