"""Pins for the oracle's SR quantities (CPU only).

P-SR1 linearity: sum_b coef_b O[b] is the batch gradient (itself pinned by finite
differences); P-SR2 per-sample scores by central differences of log pi; P-SR3 the exact
score has zero mean under pi (enumeration of all 2^n strings); P-SR4 the Fisher identity
E_pi[grad lp grad lp^T] = -E_pi[hess lp] with the Hessian by finite differences;
P-SR5 the Woodbury form equals the d x d solve, for B < d and B > d; P-SR6 the Gram is
symmetric positive semi-definite with the squared score norms on its diagonal; P-SR7 the
push-through form from the coefficients equals the d x d solve with g = O^T c; P-SR8 the
batch Fisher matrix's quadratic forms v^T I v against (1/B) sum_b (d/de log pi(s_b;
theta + e v))^2 with the directional derivatives by central differences of log pi."""
import numpy as np
import pytest

from oracle import estimator, exact, made, sr
from paper_2106_13308_amd import inputs


def _params(n, h, seed):
    p = inputs.made_init(n, h, seed)
    return {k: (v.astype(np.float64) if k != "degrees" else v) for k, v in p.items()}


def test_PSR1_linearity_against_batch_gradient():
    n, h, B = 9, 7, 13
    p = _params(n, h, 3)
    S = inputs.random_spins(B, n, 4)
    coef = np.random.default_rng(5).standard_normal(B)
    O = sr.score_matrix(p, S)
    assert O.shape == (B, n * h + h + n)                    # exactly nh unmasked weights
    assert np.allclose(coef @ O, sr.flatten(p, estimator.logp_grad(p, S, coef)), rtol=1e-12, atol=1e-13)


def test_PSR2_scores_by_central_differences():
    n, h = 6, 5
    p = _params(n, h, 11)
    s = inputs.random_spins(1, n, 12)
    O = sr.score_matrix(p, s)[0]
    M1, M2 = made.masks(n, p["degrees"])
    eps = 1e-6
    fd = {}
    for name in ("W1", "b1", "W2", "b2"):
        g = np.zeros_like(p[name])
        for idx in np.ndindex(p[name].shape):
            q = {k: (v.copy() if k != "degrees" else v) for k, v in p.items()}
            q[name][idx] += eps
            up = made.logp(q, s)[0]
            q[name][idx] -= 2 * eps
            dn = made.logp(q, s)[0]
            g[idx] = (up - dn) / (2 * eps)
        fd[name] = g
    assert np.abs(fd["W1"][M1 == 0]).max() < 1e-9 and np.abs(fd["W2"][M2 == 0]).max() < 1e-9
    assert np.allclose(O, sr.flatten(p, fd), atol=1e-7)


def test_PSR3_exact_score_has_zero_mean():
    n, h = 8, 6
    p = _params(n, h, 21)
    X = exact.all_strings(n)
    pi = np.exp(exact.log_probs(p, n))
    O = sr.score_matrix(p, X)
    assert abs(pi.sum() - 1) < 1e-12
    mean = pi @ O
    assert np.abs(mean).max() < 1e-12 * max(1.0, np.abs(O).max())
    assert np.abs(O).max() > 0.1                             # not trivially zero


def test_PSR4_fisher_identity_against_fd_hessian():
    n, h = 4, 3
    p = _params(n, h, 31)
    X = exact.all_strings(n)
    pi = np.exp(exact.log_probs(p, n))
    O = sr.score_matrix(p, X)
    I_exact = (O * pi[:, None]).T @ O                       # E_pi[grad lp grad lp^T]
    # -E_pi[hess lp]: differentiate G(theta) = sum_x pi_fixed(x) grad lp(x; theta)
    M1, M2 = made.masks(n, p["degrees"])
    cols, eps = [], 1e-5
    for name, mask in (("W1", M1), ("b1", None), ("W2", M2), ("b2", None)):
        for idx in np.ndindex(p[name].shape):
            if mask is not None and mask[idx] == 0:
                continue
            q = {k: (v.copy() if k != "degrees" else v) for k, v in p.items()}
            q[name][idx] += eps
            up = sr.flatten(p, estimator.logp_grad(q, X, pi))
            q[name][idx] -= 2 * eps
            dn = sr.flatten(p, estimator.logp_grad(q, X, pi))
            cols.append((up - dn) / (2 * eps))
    H = np.stack(cols, axis=1)
    assert H.shape == I_exact.shape
    assert np.allclose(-H, I_exact, atol=2e-6 * np.abs(I_exact).max())


@pytest.mark.parametrize("B", [5, 60])
def test_PSR5_woodbury_equals_direct_solve(B):
    n, h = 6, 4                                               # d = 24 + 4 + 6 = 34
    p = _params(n, h, 41)
    S = inputs.random_spins(B, n, 42)
    g = np.random.default_rng(43).standard_normal(n * h + h + n)
    for lam in (1e-3, 0.5):
        x1 = sr.sr_direction(p, S, g, lam)
        x2 = sr.sr_direction_woodbury(p, S, g, lam)
        assert np.allclose(x1, x2, rtol=1e-7, atol=1e-7 * np.abs(x1).max())
        # residual of the system as written
        O = sr.score_matrix(p, S)
        r = O.T @ (O @ x1) / B + lam * x1 - g
        assert np.abs(r).max() < 1e-8 * np.abs(g).max()


def test_PSR6_gram_psd_with_score_norms_on_diagonal():
    n, h, B = 10, 8, 24
    p = _params(n, h, 51)
    S = inputs.random_spins(B, n, 52)
    K = sr.gram(p, S)
    O = sr.score_matrix(p, S)
    assert np.array_equal(K, K.T) or np.allclose(K, K.T, rtol=0, atol=1e-13)
    assert np.allclose(np.diag(K), (O ** 2).sum(axis=1), rtol=1e-13)
    assert np.linalg.eigvalsh(K).min() > -1e-10 * np.abs(K).max()


@pytest.mark.parametrize("B", [5, 60])
def test_PSR7_push_through_from_coefficients_equals_direct_solve(B):
    n, h = 6, 4                                               # d = 34
    p = _params(n, h, 61)
    S = inputs.random_spins(B, n, 62)
    coef = np.random.default_rng(63).standard_normal(B) / B
    g = sr.flatten(p, estimator.logp_grad(p, S, coef))      # the batch gradient O^T c
    for lam in (1e-3, 0.5):
        x1 = sr.sr_direction(p, S, g, lam)
        x2 = sr.sr_direction_coef(p, S, coef, lam)
        assert np.allclose(x2, x1, rtol=0, atol=1e-8 * np.abs(x1).max())


def test_PSR8_fisher_quadratic_forms_by_directional_differences():
    n, h, B = 7, 5, 9
    p = _params(n, h, 71)
    S = inputs.random_spins(B, n, 72)
    I = sr.fisher(p, S)
    M1, M2 = made.masks(n, p["degrees"])
    rng = np.random.default_rng(73)
    eps = 1e-6
    for _ in range(3):
        v = {k: rng.standard_normal(np.shape(p[k])) for k in ("W1", "b1", "W2", "b2")}
        v["W1"] *= M1
        v["W2"] *= M2
        up = {k: (p[k] + eps * v[k] if k in v else p[k]) for k in p}
        dn = {k: (p[k] - eps * v[k] if k in v else p[k]) for k in p}
        dd = (made.logp(up, S) - made.logp(dn, S)) / (2 * eps)   # one directional derivative per sample
        vf = sr.flatten(p, v)
        assert np.isclose(vf @ I @ vf, (dd ** 2).mean(), rtol=1e-7)
