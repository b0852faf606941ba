"""Pins of the oracle's Algs. 5-7 and the best-of-four choice of Alg. 3's
coefficient steps (Sec. 3.2), each against a closed form or a library
least-squares routine."""
import numpy as np
import pytest

import synth
from oracle.rid import (Config, OnlineRID, alg7_transform, coeff_alg4, coeff_alg5, coeff_alg6, coeff_alg7,
                        unchanged_slots)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_alg6_as_printed_equals_alg4():
    # the algorithm box fits the residual with every basis column: P_prev +
    # S_J^+ (S - S_J P_prev) = S_J^+ S whenever S_J has full column rank
    rng = np.random.default_rng(1)
    ell, n_prev, t = 30, 40, 12
    S = rng.standard_normal((ell, n_prev + 10))
    J = np.array([3, 7, -1, 12, 20, 1, 33, 41, -1, 9, 15, 44])
    J_prev = np.array([3, 8, 5, 12, -1, 1, 30, 41, 2, 9, 16, 44])
    P_prev = rng.standard_normal((t, n_prev))
    P6 = coeff_alg6(S, J, J_prev, P_prev, literal=True)
    P4 = coeff_alg4(S, J)[:, :n_prev]
    assert _rel(P6, P4) < 1e-12


def test_alg6_keeps_the_unchanged_coefficients_and_fits_the_new_slots():
    # the old columns are the kept basis part plus an exact combination of the
    # two new basis columns: the residual fit recovers that combination
    rng = np.random.default_rng(2)
    ell, n_prev, t = 30, 40, 8
    S = rng.standard_normal((ell, n_prev + 10))          # basis columns at 40..49
    J_prev = np.arange(40, 48)
    J = np.array([40, 41, 48, 43, 49, 45, -1, 47])      # slots 2, 4 refilled, 6 emptied
    keep = unchanged_slots(J, J_prev)
    assert keep.tolist() == [True, True, False, True, False, True, False, True]
    P_prev = rng.standard_normal((t, n_prev))
    assert np.array_equal(coeff_alg6(S, J_prev, J_prev, P_prev), P_prev)   # nothing changed
    X = rng.standard_normal((2, n_prev))
    S[:, :n_prev] = S[:, J[keep]] @ P_prev[keep] + S[:, [48, 49]] @ X
    P6 = coeff_alg6(S, J, J_prev, P_prev)
    want = np.zeros((t, n_prev))
    want[keep] = P_prev[keep]
    want[[2, 4]] = X
    assert _rel(P6, want) < 1e-12


def test_alg5_with_an_isometric_sketch_is_the_exact_least_squares():
    # Omega = sqrt(l) Q^T with Q orthonormal (l >= m): Omega^T Omega = l I, so
    # Y / l = A_J^T A and P = G^{-1} A_J^T A, the least-squares coefficients
    rng = np.random.default_rng(3)
    m, n, ell = 30, 25, 40
    A = rng.standard_normal((m, n))
    Q, _ = np.linalg.qr(rng.standard_normal((ell, ell)))
    Om = np.sqrt(ell) * Q[:, :m]
    S = Om @ A
    J = np.array([2, 5, 11, -1, 19, 7])
    occ = J >= 0
    G = np.zeros((6, 6))
    G[np.ix_(occ, occ)] = A[:, J[occ]].T @ A[:, J[occ]]
    P5 = coeff_alg5(S, J, G, ell)
    want = np.linalg.lstsq(A[:, J[occ]], A, rcond=None)[0]
    assert _rel(P5[occ], want) < 1e-12
    assert np.array_equal(P5[~occ], np.zeros((1, n)))


def test_alg7_transform_is_the_least_squares_of_the_previous_basis():
    rng = np.random.default_rng(4)
    m, t = 200, 6
    C = rng.standard_normal((m, t))
    C_prev = C.copy()
    C_prev[:, 1] = rng.standard_normal(m)         # slot 1 held another column before
    C_prev[:, 4] = C @ rng.standard_normal(t)     # and slot 4 a column inside span(C)
    J = np.arange(t)
    J_prev = np.arange(t) + np.array([0, 100, 0, 0, 200, 0])
    T = alg7_transform(C, J, C_prev, J_prev)
    want = np.linalg.lstsq(C, C_prev, rcond=None)[0]
    assert _rel(T, want) < 1e-12
    # unchanged slots map to themselves; a previous column inside the span is
    # reproduced exactly
    assert np.allclose(T[:, [0, 2, 3, 5]], np.eye(t)[:, [0, 2, 3, 5]], atol=1e-12)
    assert np.allclose(C @ T[:, 4], C_prev[:, 4], atol=1e-10 * np.abs(C_prev[:, 4]).max())
    P_prev = rng.standard_normal((t, 30))
    assert np.allclose(coeff_alg7(T, P_prev), T @ P_prev)


@pytest.fixture(scope="module")
def best4_run():
    A = synth.lowrank(6000, 300, seed=3, rank=60, rel_noise=1e-3)
    o = OnlineRID(Config(m=6000, ell=40, k=20, t=20, coeff="best4", omega_seed=5, select_seed=6), n_max=300)
    o.push(A.T)
    o.finalize()
    return A, o


def test_best_of_four_keeps_the_smallest_estimate(best4_run):
    _, o = best4_run
    qs = [r.q_star for r in o.records]
    for r in o.records:
        e = np.array(r.e2_q)
        assert r.q_star == 4 + int(np.flatnonzero(e == e.min())[0])   # ties: the lowest q
        assert r.hutch["E2"] == e.min()
    # with nothing before it, Algs. 6 and 7 are Alg. 4 at the first update
    e0 = o.records[0].e2_q
    assert e0[0] == e0[2] == e0[3]
    assert len(set(qs)) > 1, qs


def test_best_of_four_never_estimates_worse_than_alg4():
    # the coefficients do not enter the selection, so both modes select the
    # same J; Alg. 4's candidate is the Alg.-4-only P of that update, so its
    # estimate is the same number, and the kept estimate is never larger
    A = synth.lowrank(4000, 160, seed=9, rank=30, rel_noise=1e-4)
    cfg = dict(m=4000, ell=40, k=20, t=20, omega_seed=7, select_seed=8)
    o4 = OnlineRID(Config(**cfg), n_max=160)
    ob = OnlineRID(Config(**cfg, coeff="best4"), n_max=160)
    for o in (o4, ob):
        o.push(A.T)
        o.finalize()
    assert np.array_equal(o4.J, ob.J)
    for r4, rb in zip(o4.records, ob.records):
        assert np.array_equal(r4.J, rb.J)
        assert rb.e2_q[0] == r4.hutch["E2"]
        assert rb.hutch["E2"] <= r4.hutch["E2"]
