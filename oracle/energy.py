"""Diagonal local energy.

For a diagonal Hamiltonian (alpha_i = 0 in eq. (hamiltonian) / eq. (e:tim)) the local
energy l(x) = (H psi)(x) / psi(x) of Sec. 2.1 is the diagonal entry H_xx.  With
beta_i = 0 and couplings J_ij this is a quadratic form in the spins s = 1 - 2x.
Reading R5 (the paper's Max-Cut sign and 1/4 factor would make the empty cut optimal):
minimise

    E(s) = sum_{i<j} J_ij s_i s_j,      and for a weighted graph J_ij = w_ij,
    cut(s) = sum_{(i,j) in E} w_ij [s_i != s_j] = (W_tot - E(s)) / 2.
"""
from __future__ import annotations

import numpy as np


def energy_edges(edges, weights, S) -> np.ndarray:
    """E_b = sum over listed edges (i, j) of w_ij s_i s_j.

    Integer weights give exact int64 results; float weights give float64."""
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = np.asarray(weights)
    S = np.asarray(S)
    if np.issubdtype(w.dtype, np.integer):
        Si = S[:, edges[:, 0]].astype(np.int64)
        Sj = S[:, edges[:, 1]].astype(np.int64)
        return (Si * Sj * w.astype(np.int64)[None, :]).sum(axis=1, dtype=np.int64)
    Si = S[:, edges[:, 0]].astype(np.float64)
    Sj = S[:, edges[:, 1]].astype(np.float64)
    return (Si * Sj * w.astype(np.float64)[None, :]).sum(axis=1)


def energy_dense(J, S) -> np.ndarray:
    """E_b = sum_{i<j} J_ij s_i s_j for a dense coupling matrix (float64)."""
    J = np.asarray(J, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    Ju = np.triu(J, 1)
    return np.einsum("bi,ij,bj->b", S, Ju, S)


def total_weight(weights):
    w = np.asarray(weights)
    return int(w.astype(np.int64).sum()) if np.issubdtype(w.dtype, np.integer) else float(w.sum())


def cut_value(edges, weights, S) -> np.ndarray:
    """Weight of edges whose endpoints carry different spins (direct definition)."""
    edges = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    S = np.asarray(S)
    diff = S[:, edges[:, 0]] != S[:, edges[:, 1]]
    return (diff * np.asarray(weights)[None, :]).sum(axis=1)
