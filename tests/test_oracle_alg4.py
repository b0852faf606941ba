"""Pins of the oracle's coefficients (Alg. 4, eq. coeff_rID_fullsketch)."""
import numpy as np

from oracle.exact import exact_error
from oracle.rid import Config, OnlineRID, coeff_alg4, pinv, sketch_columns


def test_interpolation_property():
    rng = np.random.default_rng(0)
    S = rng.standard_normal((30, 80))
    J = np.array([3, 70, 12, 44, 5, 61])
    P = coeff_alg4(S, J)
    assert np.allclose(P[:, J], np.eye(6), atol=1e-12)


def test_exact_recovery_for_data_in_the_span_of_the_basis():
    # A = A_J X  =>  P = X for any Omega (the sketched LS is then exact)
    rng = np.random.default_rng(1)
    m, n, t = 400, 40, 5
    J = np.array([2, 9, 17, 30, 38])
    AJ = rng.standard_normal((m, t))
    X = rng.standard_normal((t, n))
    X[:, J] = np.eye(t)
    A = AJ @ X
    for seed in (1, 2):
        S, _ = sketch_columns(A, seed, 12)
        P = coeff_alg4(S, J)
        assert np.allclose(P, X, atol=1e-9)


def test_equals_library_least_squares():
    rng = np.random.default_rng(2)
    S = rng.standard_normal((24, 50))
    J = np.array([1, 4, 9, 16, 25, 36, 49, 0])
    P = coeff_alg4(S, J)
    ref = np.linalg.lstsq(S[:, J], S, rcond=None)[0]
    assert np.allclose(P, ref, atol=1e-11)


def test_empty_slots_get_zero_rows():
    rng = np.random.default_rng(3)
    S = rng.standard_normal((16, 30))
    J = np.array([4, -1, 8, -1, 20])
    P = coeff_alg4(S, J)
    assert np.all(P[[1, 3]] == 0)
    ref = np.linalg.lstsq(S[:, [4, 8, 20]], S, rcond=None)[0]
    assert np.allclose(P[[0, 2, 4]], ref, atol=1e-11)


def test_pinv_matches_library_on_rank_deficient_input():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((20, 4)) @ rng.standard_normal((4, 9))
    assert np.allclose(pinv(a), np.linalg.pinv(a), atol=1e-10)


def test_zero_error_when_every_column_is_kept():
    # n <= t: the only update keeps every column, A_J P reproduces A
    rng = np.random.default_rng(5)
    m, n, t = 300, 6, 8
    A = rng.standard_normal((m, n))
    # l = 32 gives n1 = 8 >= rank(A) = 6, so the estimate is exact as well
    cfg = Config(m=m, ell=32, k=t, t=t, omega_seed=3, select_seed=4)
    o = OnlineRID(cfg)
    o.push(A)
    o.finalize()
    assert sorted(o.J[o.J >= 0]) == list(range(n))
    assert exact_error(A, o.J, o.P) <= 1e-10 * np.linalg.norm(A)
    assert abs(o.records[-1].hutch["E2"]) <= 1e-9 * o.F
