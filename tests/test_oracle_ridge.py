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
    sk2, _, mu = ridge_lambda(SST, 0.0, 5, 20, 1e-8)
    F = 3.7
    _, lam, _ = ridge_lambda(SST, F, 5, 20, 1e-8)
    tail = float(np.sum(mu[5:]))
    assert np.isclose(lam, F * tail / float(np.sum(mu)) / 5, rtol=1e-12)
    # the sketch's rank is <= k: its tail is zero and the floor holds
    S = _sketch(rng, 20, 40, 4)
    _, lam, _ = ridge_lambda(S @ S.T, F, 5, 20, 1e-8)
    assert lam == 1e-8 * F / 5


def test_lambda_is_the_rank_k_tail_for_an_isometric_sketch():
    # eq. ridge-leverage-score sets lam = ||A - A_k||_F^2 / k.  When Omega / sqrt(l)
    # acts as an isometry on the range of A (Omega = sqrt(l) Q^T with Q an
    # orthonormal basis of a space holding range(A)), the reading returns
    # exactly that value, whatever the scale of the sketch.
    rng = np.random.default_rng(5)
    m, n, ell, k = 200, 60, 30, 7
    A = rng.standard_normal((m, 25)) @ np.diag(0.8 ** np.arange(25)) @ rng.standard_normal((25, n))
    Q, _ = np.linalg.qr(np.hstack([np.linalg.qr(A)[0][:, :25], rng.standard_normal((m, ell - 25))]))
    sv = np.linalg.svd(A, compute_uv=False)
    F = float(np.sum(A * A))
    want = float(np.sum(sv[k:] ** 2)) / k
    for scale in (1.0, 7.5):
        S = scale * np.sqrt(ell) * Q.T @ A
        _, lam, _ = ridge_lambda(S @ S.T, F, k, ell, 1e-8)
        assert np.isclose(lam, want, rtol=1e-10)


def test_lambda_tracks_the_tail_where_the_difference_of_estimates_fails():
    # A Gaussian sketch of a matrix whose energy sits in a few directions:
    # ||S||^2 / l fluctuates around F by far more than the rank-k tail, so the
    # printed form with ||S_k||^2 / l in place of the sketch's own top-k
    # fraction swings from negative (then the floor) to many times the tail.
    # The tail fraction of the sketch itself stays near the true
    # ||A - A_k||_F^2 / k on every seed.
    m, n, ell, k = 2000, 200, 100, 20
    negative = 0
    for seed in range(10):
        rng = np.random.default_rng(seed)
        U = np.linalg.qr(rng.standard_normal((m, n)))[0]
        V = np.linalg.qr(rng.standard_normal((n, n)))[0]
        sv = 0.85 ** np.arange(n)
        A = (U * sv) @ V.T
        F = float(np.sum(sv ** 2))
        S = rng.standard_normal((ell, m)) @ A
        sk2, lam, _ = ridge_lambda(S @ S.T, F, k, ell, 1e-8)
        true = float(np.sum(sv[k:] ** 2)) / k
        assert 0.5 * true < lam < 1.2 * true
        negative += (F - sk2 / ell) < 0.0
    assert negative >= 3


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
