"""Pins of the oracle's Gaussian test matrix Omega (Alg. 3 step 2)."""
import math

import numpy as np
import scipy.stats as st
import torch

from scipy.special import ndtr, ndtri

from oracle.omega import (omega_block, omega_bound, omega_entry_scalar, omega_from_halves, omega_scale, omega_table,
                          round_to_bf16)


def test_block_matches_scalar_brute_force():
    ell, m = 19, 23
    blk = omega_block(4242, ell, 0, m)
    for r in range(ell):
        for i in range(m):
            assert abs(blk[r, i] - omega_entry_scalar(4242, r, i)) <= 1e-15 * (1 + abs(blk[r, i]))


def test_high_counter_word():
    i0 = (1 << 32) + 5
    blk = omega_block(7, 8, i0, 3)
    for r in range(8):
        for d in range(3):
            assert blk[r, d] == omega_entry_scalar(7, r, i0 + d)


def test_blocks_are_consistent():
    full = omega_block(11, 30, 100, 50)
    part = np.concatenate([omega_block(11, 30, 100, 17), omega_block(11, 30, 117, 33)], axis=1)
    assert np.array_equal(full, part)
    # the first rows of a taller Omega are the rows of a shorter one
    assert np.array_equal(omega_block(11, 40, 100, 50)[:30], full)


def test_table_holds_the_half_normal_quantiles():
    # Phi(T[k] / c) must be the middle of the k-th of 1024 equiprobable bins
    # of |N(0,1)|; checked through the forward CDF (an independent routine)
    T = omega_table()
    c = omega_scale()
    assert T.shape == (1024,) and np.all(np.diff(T) > 0) and T[0] > 0
    k = np.arange(1024)
    p = 0.5 * (1.0 + (k + 0.5) / 1024)
    assert np.max(np.abs(ndtr(T / c) - p)) < 1e-15
    # quantising at bin midpoints loses a little variance; c puts it back
    assert 1.0 < c < 1.001


def test_entries_have_mean_zero_and_exactly_unit_variance():
    # Sec. 3.3: mean 0, variance 1.  Over all 2^16 halves every table entry
    # appears 64 times with each sign, so these are the exact moments of an
    # entry of Omega.
    h = np.arange(1 << 16)
    z = omega_from_halves(h)
    assert z.sum() == 0.0
    assert abs(np.mean(z * z) - 1.0) < 1e-15
    counts = np.unique(z, return_counts=True)[1]
    assert counts.size == 2048 and np.all(counts == 32)


def test_distribution_is_within_one_atom_of_the_normal():
    # the CDF of the 2048 equiprobable atoms against Phi: at most the 1/2048
    # jump at an atom plus the small outward shift of the scale c
    T = omega_table()
    atoms = np.concatenate([-T[::-1], T])
    F_after = np.arange(1, 2049) / 2048.0
    F_before = np.arange(0, 2048) / 2048.0
    Phi = ndtr(atoms)
    d = max(np.max(np.abs(F_after - Phi)), np.max(np.abs(F_before - Phi)))
    assert d < 0.6 / 1024


def test_entry_bound():
    # the largest magnitude is the top quantile, Phi^{-1}(1 - 1/4096) scaled
    assert abs(omega_bound() - omega_scale() * float(ndtri(1.0 - 0.25 / 1024))) < 1e-14
    assert 3.4 < omega_bound() < 3.6


def test_moments_and_normality():
    z = omega_block(2024, 64, 0, 32768).ravel()
    n = z.size
    assert abs(z.mean()) < 4.0 / math.sqrt(n)
    # Var of the sample variance of a normal: 2 sigma^4 / n
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    # the atoms' fourth moment (the tails beyond 3.49 are folded into the
    # outermost atoms, so it is slightly below the normal's 3)
    k4 = float(np.mean(omega_table() ** 4))
    assert 2.97 < k4 < 3.0
    kurt = np.mean(z ** 4) / z.var() ** 2
    assert abs(kurt - k4) < 4.0 * math.sqrt(24.0 / n)
    assert np.max(np.abs(z)) <= omega_bound()
    d = st.kstest(z[:400000], "norm").statistic
    assert d < 1.63 / math.sqrt(400000)


def test_rows_are_uncorrelated():
    blk = omega_block(5, 16, 0, 100000)
    c = np.corrcoef(blk)
    off = c[~np.eye(16, dtype=bool)]
    assert np.max(np.abs(off)) < 4.5 / math.sqrt(100000)


def test_bf16_rounding_matches_library():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0]]).astype(np.float32)
    lib = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(round_to_bf16(x), lib)
