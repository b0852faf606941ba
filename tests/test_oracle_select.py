"""Pins of the oracle's prune/fill step (Alg. 3 inner loop over slots)."""
import math

import numpy as np

import synth
from oracle.philox import PRUNE_DRAW, decision_uniform
from oracle.rid import Config, OnlineRID, fill_factor, select_slots


def test_unchanged_scores_never_prune():
    t = 8
    J = np.arange(t) * 3
    tau = np.linspace(0.1, 0.9, t)
    J2, tau2, filled, dec = select_slots(0, J, tau, tau.copy(), np.ones(4), [100, 101, 102, 103], 10.0, 5)
    assert np.array_equal(J2, J) and not filled.any()
    assert all(d.p == 0.0 and not d.success for d in dec)


def test_certain_fill_takes_buffer_in_order():
    t = 6
    J = np.full(t, -1)
    d_idx = [10, 11, 12, 13, 14, 15, 16]
    J2, tau2, filled, _ = select_slots(0, J, np.ones(t), np.full(t, np.nan), np.ones(7), d_idx, 1.0, 3)
    assert list(J2) == d_idx[:t]
    assert filled.all() and np.all(tau2 == 1.0)


def test_zero_scores_prune_everything_and_fill_nothing():
    t = 5
    J = np.arange(t)
    J2, tau2, filled, _ = select_slots(1, J, np.ones(t), np.zeros(t), np.zeros(3), [7, 8, 9], 10.0, 3)
    assert np.all(J2 == -1) and np.all(tau2 == 1.0) and not filled.any()


def test_no_buffer_column_is_placed_twice():
    rng = np.random.default_rng(0)
    for s in range(50):
        t = 10
        J = np.where(rng.random(t) < 0.5, rng.integers(0, 50, t), -1)
        tau_old = rng.uniform(0.2, 1.0, t)
        tau_C = tau_old * rng.uniform(0.0, 1.0, t)
        tau_D = rng.uniform(0, 0.2, t)
        J2, _, filled, _ = select_slots(s, J, tau_old, tau_C, tau_D, list(range(100, 110)), 5.0, s)
        new = J2[filled]
        assert len(set(new)) == len(new)


def test_prune_frequency_matches_probability():
    # "with probability 1 - tau/tau_old": empirical frequency over many updates
    p = 0.3
    n = 20000
    hits = 0
    for u in range(n // 50):
        J2, _, _, _ = select_slots(u, np.arange(50), np.ones(50), np.full(50, 1 - p),
                                   np.zeros(0), [], 1.0, 17)
        hits += int(np.sum(J2 < 0))
    assert abs(hits / n - p) < 4 * math.sqrt(p * (1 - p) / n)


def test_fill_scan_first_success_frequency():
    # one empty slot, constant q: the filled position is geometric in r
    q = 0.25
    pos = []
    for u in range(4000):
        J2, _, _, _ = select_slots(u, np.array([-1]), np.ones(1), np.full(1, np.nan),
                                   np.full(8, q), list(range(8)), 1.0, 23)
        pos.append(J2[0])
    pos = np.array(pos)
    for r in range(3):
        pr = q * (1 - q) ** r
        assert abs(np.mean(pos == r) - pr) < 4 * math.sqrt(pr * (1 - pr) / len(pos))
    assert abs(np.mean(pos == -1) - (1 - q) ** 8) < 4 * math.sqrt((1 - q) ** 8 / len(pos))


def test_prune_draw_uses_its_own_counter():
    t = 3
    tau_old = np.ones(t)
    tau_C = np.full(t, 0.5)
    _, _, _, dec = select_slots(4, np.arange(t), tau_old, tau_C, np.zeros(0), [], 1.0, 99)
    for d in dec:
        assert d.U == float(decision_uniform(99, 4, d.slot, PRUNE_DRAW))


def test_stream_first_update_takes_first_columns_and_F_is_exact():
    # with q saturated at 1 (fill factor * tau >= 1) the first update keeps
    # the first t columns; F accumulates every pushed column (no column skipped)
    A = synth.sines(512, 64, seed=1).T
    cfg = Config(m=512, ell=16, k=8, t=8, omega_seed=5, select_seed=6)
    o = OnlineRID(cfg)
    o.push(A[:, :8])
    rec = o.records[0]
    assert np.all(np.minimum(1, o.fill_mult * rec.tau_D) == 1.0)
    assert list(o.J) == list(range(8))
    o.push(A[:, 8:])
    assert math.isclose(o.F, math.fsum((A.astype(np.float64) ** 2).ravel()), rel_tol=1e-13)
    assert len(o.records) == 8


def test_fill_factor_hand_values():
    # Alg. 3 fill step: c (k log k + k log(1/delta) / eps) / t with the natural
    # log.  Evaluated by hand with k != t: (10 ln 10 + 10 ln 20 / 0.5) / 25
    # = (23.02585 + 59.91465) / 25 = 3.317620.
    cfg = Config(m=1, ell=40, k=10, t=25, delta=0.05, eps=0.5, c_sample=1.0)
    assert abs(fill_factor(cfg) - 3.317620) < 1e-6
    # c multiplies; delta and eps enter only through ln(1/delta) / eps
    assert abs(fill_factor(Config(m=1, ell=40, k=10, t=25, c_sample=2.5)) - 2.5 * 3.317620) < 1e-5
    cfg = Config(m=1, ell=40, k=10, t=25, delta=0.01, eps=0.25)
    assert abs(fill_factor(cfg) - (23.02585 + 10 * 4.605170 / 0.25) / 25) < 1e-5
    # k = t: ln k + 2 ln 20 at delta = 0.05, eps = 0.5 (alpha of the five
    # workloads: l = 40, 200, 300, 200, 400 with k = t = l / 2)
    for k, alpha in ((20, 8.99), (100, 10.60), (150, 11.00), (200, 11.29)):
        assert abs(fill_factor(Config(m=1, ell=2 * k, k=k, t=k)) - alpha) < 0.005


def test_fill_frequency_follows_the_fill_factor():
    # one empty slot, one buffered column with score tau: it is filled with
    # probability alpha tau (k = 10, t = 25: alpha = 3.3176, tau = 0.1)
    cfg = Config(m=1, ell=40, k=10, t=25)
    a = fill_factor(cfg)
    tau = 0.1
    n = 6000
    hits = 0
    for u in range(n):
        J2, _, _, _ = select_slots(u, np.array([-1]), np.ones(1), np.full(1, np.nan),
                                   np.full(1, tau), [0], a, 31)
        hits += int(J2[0] == 0)
    p = a * tau
    assert abs(hits / n - p) < 4 * math.sqrt(p * (1 - p) / n)
