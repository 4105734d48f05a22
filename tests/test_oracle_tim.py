"""Pins for the oracle's TIM local energy (CPU only).

P-TIM1 the entries the oracle uses (diagonal, -alpha_i at single flips, zero elsewhere) equal
those of H built from its definition as Kronecker products of Pauli matrices, for every
pair of strings (pins signs, the s = 1 - 2x map and the bit order); P-TIM2 the local energy
equals (H psi)(x) / psi(x) with psi = sqrt(pi) over all strings; P-TIM3 its pi-average is
<psi|H|psi> and is >= the smallest eigenvalue (variational inequality); P-TIM4 closed forms:
independent sites (no weights) give the log-ratio -s_i b2_i, and the uniform state is the
ground state of the pure transverse field, with local energy -sum alpha_i everywhere; P-TIM5 the last site's flip
only changes its own conditional."""
import numpy as np
import pytest

from oracle import exact, made, tim
from paper_2106_13308_amd import inputs


def _params(n, h, seed, scale=2.0):
    p = inputs.made_init(n, h, seed)
    p["W1"] = p["W1"] * scale
    p["W2"] = p["W2"] * scale
    return {k: (v.astype(np.float64) if k != "degrees" else v) for k, v in p.items()}


def test_PTIM1_entries_match_pauli_definition():
    n = 4
    c = inputs.tim_couplings(n, 3)
    H = tim.hamiltonian_dense(c["alpha"], c["beta"], c["beta_ij"])
    X = exact.all_strings(n)                                  # row index x -> spins
    assert np.allclose(np.diag(H), tim.diag_energy(c["beta"], c["beta_ij"], X), rtol=0, atol=1e-12)
    N = 2 ** n
    for x in range(N):
        for y in range(N):
            if x == y:
                continue
            diff = x ^ y
            if diff & (diff - 1) == 0:                         # one bit apart
                i = n - 1 - int(np.log2(diff))                 # site 0 is the most significant bit
                assert H[x, y] == pytest.approx(-float(c["alpha"][i]), abs=1e-12)
            else:
                assert H[x, y] == 0.0


def test_PTIM2_local_energy_equals_H_psi_over_psi():
    n, h = 8, 10
    p = _params(n, h, 5)
    c = inputs.tim_couplings(n, 6)
    X = exact.all_strings(n)
    pi = np.exp(exact.log_probs(p, n))
    psi = np.sqrt(pi)
    H = tim.hamiltonian_dense(c["alpha"], c["beta"], c["beta_ij"])
    ref = (H @ psi) / psi
    got = tim.local_energy(p, X, c["alpha"], c["beta"], c["beta_ij"])
    assert np.allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_PTIM3_average_is_rayleigh_quotient_and_variational():
    n, h = 8, 12
    p = _params(n, h, 7)
    c = inputs.tim_couplings(n, 8)
    X = exact.all_strings(n)
    pi = np.exp(exact.log_probs(p, n))
    H = tim.hamiltonian_dense(c["alpha"], c["beta"], c["beta_ij"])
    L = pi @ tim.local_energy(p, X, c["alpha"], c["beta"], c["beta_ij"])
    psi = np.sqrt(pi)
    assert L == pytest.approx(psi @ H @ psi, rel=1e-12)
    assert L >= np.linalg.eigvalsh(H).min() - 1e-12


def test_PTIM4_closed_forms():
    n, h = 9, 7
    p = _params(n, h, 9)
    S = inputs.random_spins(16, n, 10)
    # independent sites (no weights): flipping site i changes only log sigma(s_i b2_i)
    q = dict(p)
    q["W1"] = np.zeros_like(p["W1"])
    q["W2"] = np.zeros_like(p["W2"])
    D = tim.flip_logratio(q, S)
    assert np.allclose(D, -S * q["b2"][None, :], rtol=0, atol=1e-12)
    # uniform state (zero weights and biases) is the ground state of -sum alpha_i X_i:
    # every string has local energy -sum alpha_i, so the variance is 0
    q["b1"] = np.zeros_like(p["b1"])
    q["b2"] = np.zeros_like(p["b2"])
    c = inputs.tim_couplings(n, 11)
    l = tim.local_energy(q, S, c["alpha"], np.zeros(n), np.zeros((n, n)))
    assert np.allclose(l, -np.sum(c["alpha"], dtype=np.float64), rtol=0, atol=1e-12)


def test_PTIM5_last_site_flip_changes_one_conditional():
    n, h = 12, 9
    p = _params(n, h, 12)
    S = inputs.random_spins(32, n, 13)
    z = made.forward(p, S)["Z"][:, n - 1]
    D = tim.flip_logratio(p, S, sites=[n - 1])[:, 0]
    # log sigma(-t) - log sigma(t) = -t with t = s_n z_n
    assert np.allclose(D, -S[:, n - 1] * z, rtol=1e-12, atol=1e-12)
