"""Pins of the oracle's NA-Hutch++ error estimate (Alg. 8; eqs. Hutchinson,
NAhutchPP1, NAhutchPP_expansion, NAhutchPP_2nd_term)."""
import math

import numpy as np

from oracle.exact import exact_ls
from oracle.omega import omega_block
from oracle.rid import nahutchpp, pinv


def _problem(seed, m=200, n=40, rank=10, t=6):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, rank)) @ (rng.standard_normal((rank, n)) * np.exp(-np.arange(rank) / 2)[:, None])
    A += 0.05 * rng.standard_normal((m, n))
    J = np.sort(rng.choice(n, t, replace=False))
    P = exact_ls(A, J) + 0.1 * rng.standard_normal((t, n))
    G = A[:, J].T @ A[:, J]
    return A, J, P, G, float(np.sum(A * A))


def test_no_low_rank_part_is_hutchinson():
    A, J, P, G, F = _problem(0)
    ell = 20
    Om = omega_block(3, ell, 0, A.shape[0])
    S = Om @ A
    B = A @ (A[:, J] @ P).T
    hutch = np.trace(Om @ B @ Om.T) / ell
    est = nahutchpp(S, S[:, J], P, G, F, 0, 0)["tr_est"]
    assert math.isclose(est, hutch, rel_tol=1e-10)


def test_sketch_only_formula_equals_explicit_na_hutchpp():
    # eq. NAhutchPP_2nd_term (sketch only) against eq. NAhutchPP1 written
    # out with the m x m matrix B = A (A_J P)^T formed explicitly
    A, J, P, G, F = _problem(1)
    ell, n1, n2 = 24, 6, 12
    n3 = ell - n1 - n2
    Om = omega_block(8, ell, 0, A.shape[0])
    O1, O2, O3 = Om[:n1], Om[n1:n1 + n2], Om[n1 + n2:]
    B = A @ (A[:, J] @ P).T
    Bt = (O2 @ B).T @ pinv(O1 @ B @ O2.T) @ (O1 @ B)
    explicit = np.trace(Bt) + (np.trace(O3 @ B @ O3.T) - np.trace(O3 @ Bt @ O3.T)) / n3
    S = Om @ A
    est = nahutchpp(S, S[:, J], P, G, F, n1, n2)["tr_est"]
    assert math.isclose(est, explicit, rel_tol=1e-8)


def test_expansion_identity():
    # ||A - A_J P||^2 = ||A||^2 - 2 tr(A (A_J P)^T) + tr(G P P^T)
    A, J, P, G, F = _problem(2)
    lhs = np.sum((A - A[:, J] @ P) ** 2)
    rhs = F - 2 * np.sum(A * (A[:, J] @ P)) + np.sum((G @ P) * P)
    assert math.isclose(lhs, rhs, rel_tol=1e-10)


def test_zero_coefficients_give_F():
    A, J, P, G, F = _problem(3)
    S = omega_block(4, 16, 0, A.shape[0]) @ A
    out = nahutchpp(S, S[:, J], np.zeros_like(P), G, F, 4, 8)
    assert out["E2"] == F


def test_exact_when_reconstruction_is_exact_and_rank_small():
    # A = A_J P exactly with rank(A) <= n1: B is symmetric of rank <= n1, the
    # Nystrom part is exact and the estimate is the true error, zero
    rng = np.random.default_rng(4)
    m, n, r = 300, 30, 4
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    J = np.array([0, 5, 11, 20])
    P = exact_ls(A, J)
    G = A[:, J].T @ A[:, J]
    F = float(np.sum(A * A))
    S = omega_block(6, 24, 0, m) @ A
    out = nahutchpp(S, S[:, J], P, G, F, 6, 12)
    assert abs(out["E2"]) <= 1e-9 * F


def test_unbiased_over_test_matrices():
    # (J, P) fixed independently of Omega: the mean over 2000 draws of Omega
    # matches the exact trace within 4 standard errors
    A, J, P, G, F = _problem(5, m=300, n=60, rank=12, t=6)
    exact = float(np.sum(A * (A[:, J] @ P)))
    ests = np.array([nahutchpp(*(lambda S: (S, S[:, J]))(omega_block(10_000 + s, 24, 0, A.shape[0]) @ A),
                               P, G, F, 6, 12)["tr_est"] for s in range(2000)])
    se = ests.std() / math.sqrt(len(ests))
    assert abs(ests.mean() - exact) < 4 * se


def test_reused_sketch_reads_the_residual_low_independent_matrix_does_not():
    # Sec. 4 queries E = A - A_J P through the rows of Omega A that Alg. 4
    # fitted P to, so the queried residual is a least-squares residual and
    # carries less than its share of ||E||_F^2; an independent Gaussian test
    # matrix reads it without that shortfall (averaged over three seeds)
    from oracle.rid import Config, OnlineRID
    m, n, ell, t = 2000, 240, 96, 48
    reused, fresh = [], []
    for seed in range(3):
        rng = np.random.default_rng(100 + seed)
        r = 150
        A = (rng.standard_normal((m, r)) / np.sqrt(1.0 + np.arange(r))) @ rng.standard_normal((r, n))
        o = OnlineRID(Config(m=m, ell=ell, k=t, t=t, omega_seed=7 + seed, select_seed=9 + seed, operand="f64"),
                      n_max=n)
        o.push(A)
        o.finalize()
        occ = o.J >= 0
        E = A - A[:, o.J[occ]] @ o.P[occ]
        exact = float(np.sum(E * E))
        W = rng.standard_normal((ell, m))
        reused.append(o.records[-1].hutch["E2"] / exact)
        fresh.append(float(np.sum((W @ E) ** 2)) / ell / exact)
    assert np.mean(reused) < 0.8, reused
    assert 0.8 < np.mean(fresh) < 1.2, fresh
