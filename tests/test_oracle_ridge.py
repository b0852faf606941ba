"""Pins of the oracle's sketched ridge leverage scores
(eq. sketch_ridge_leverage_score; Alg. 3 function)."""
import numpy as np

from oracle.rid import ridge_lambda, ridge_scores


def _sketch(rng, ell, n, rank):
    return rng.standard_normal((ell, rank)) @ rng.standard_normal((rank, n))


def test_explicit_inverse_small():
    rng = np.random.default_rng(0)
    for ell in (4, 6, 8):
        S = _sketch(rng, ell, 12, 3)
        SST = S @ S.T
        F = float(np.sum(S * S)) / ell * 1.3
        sk2, lam, _ = ridge_lambda(SST, F, 2, ell, 1e-8)
        tau = ridge_scores(SST, lam, ell, S)
        Minv = np.linalg.inv(SST + ell * lam * np.eye(ell))
        brute = np.array([S[:, j] @ Minv @ S[:, j] for j in range(S.shape[1])])
        assert np.allclose(tau, brute, rtol=1e-10, atol=0)


def test_top_k_energy_from_singular_values():
    rng = np.random.default_rng(1)
    S = _sketch(rng, 30, 50, 12) + 0.01 * rng.standard_normal((30, 50))
    for k in (1, 5, 12, 29, 30, 45):
        sk2, _, _ = ridge_lambda(S @ S.T, 1.0, k, 30, 1e-8)
        sv = np.linalg.svd(S, compute_uv=False)
        assert np.isclose(sk2, np.sum(sv[:min(k, 30)] ** 2), rtol=1e-12)


def test_lambda_formula_and_floor():
    rng = np.random.default_rng(2)
    S = _sketch(rng, 20, 40, 20)
    SST = S @ S.T
    sk2, _, _ = ridge_lambda(SST, 0.0, 5, 20, 1e-8)
    F = 2.0 * sk2 / 20
    _, lam, _ = ridge_lambda(SST, F, 5, 20, 1e-8)
    assert np.isclose(lam, (F - sk2 / 20) / 5, rtol=1e-14)
    F = 0.5 * sk2 / 20                       # tail estimate negative -> floor
    _, lam, _ = ridge_lambda(SST, F, 5, 20, 1e-8)
    assert lam == 1e-8 * F / 5


def test_sum_of_scores_closed_form_and_bounds():
    # sum_j s_j^T M^{-1} s_j = tr(M^{-1} SS^T) = sum_r mu_r / (mu_r + l lam)
    rng = np.random.default_rng(3)
    ell = 24
    S = _sketch(rng, ell, 60, 10) + 0.1 * rng.standard_normal((ell, 60))
    SST = S @ S.T
    F = float(np.sum(S * S)) / ell
    sk2, lam, mu = ridge_lambda(SST, F, 6, ell, 1e-8)
    tau = ridge_scores(SST, lam, ell, S)
    assert np.isclose(tau.sum(), np.sum(mu / (mu + ell * lam)), rtol=1e-10)
    assert np.all(tau >= 0) and np.all(tau <= 1)


def test_monotone_when_a_column_is_added():
    # At a fixed ridge, adding a column to the observed matrix can only lower
    # the scores of the columns already observed (the monotonicity that
    # Sec. 2.2.2 states in words).
    rng = np.random.default_rng(4)
    ell = 16
    S = _sketch(rng, ell, 30, 8)
    b = rng.standard_normal(ell)
    lam = 0.3
    tau0 = ridge_scores(S @ S.T, lam, ell, S)
    tau1 = ridge_scores(S @ S.T + np.outer(b, b), lam, ell, S)
    assert np.all(tau1 <= tau0 * (1 + 1e-12))
