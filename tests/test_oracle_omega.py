"""Pins of the oracle's Gaussian test matrix Omega (Alg. 3 step 2)."""
import math

import numpy as np
import scipy.stats as st
import torch

from oracle.omega import _box_muller, omega_block, omega_bound, omega_entry_scalar, omega_variance, round_to_bf16


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


def test_variance_closed_form():
    # the plain 16-bit transform: E[R^2]/2 summed directly over the u1 grid
    n = 1 << 16
    direct = float(np.mean(-np.log((np.arange(n) + 1.0) / n)))
    assert abs(omega_variance() - direct) < 1e-12
    assert abs(omega_variance() - (1.0 - 9.87e-5)) < 1e-6


def test_entries_have_exactly_unit_variance():
    # Sec. 3.3: the test matrix has mean-0, variance-1 entries.  Through the
    # generator's own transform: for a fixed 16-bit angle, cos^2 + sin^2 = 1,
    # so the mean of (z0^2 + z1^2) / 2 over every 16-bit radius word is the
    # exact second moment of an entry (the angle averages cos^2 and sin^2 to
    # 1/2 each, exactly, over its 2^16 equispaced values).
    for hi in (0, 1, 12345, 65535):
        words = (np.arange(1 << 16, dtype=np.uint64) | np.uint64(hi << 16))
        w4 = np.stack([words, words, words, words], axis=-1)
        z = _box_muller(w4)
        m2 = float(np.mean((z[:, 0] ** 2 + z[:, 1] ** 2) / 2.0))
        assert abs(m2 - 1.0) < 1e-13
    ang = np.arange(1 << 16) / 65536.0
    assert abs(np.mean(np.cos(2 * np.pi * ang) ** 2) - 0.5) < 1e-14
    assert abs(np.mean(np.cos(2 * np.pi * ang))) < 1e-14


def test_entry_bound():
    # the largest radius comes from u1 = 1/N: sqrt(2 ln N / v) = 4.7098
    assert abs(omega_bound() - 4.7098) < 1e-4
    z = _box_muller(np.array([[0, 0, 0, 0]], dtype=np.uint64))
    assert abs(z[0, 0] - omega_bound()) < 1e-15 * omega_bound()


def test_moments_and_normality():
    z = omega_block(2024, 64, 0, 32768).ravel()
    n = z.size
    assert abs(z.mean()) < 4.0 / math.sqrt(n)
    # Var of the sample variance of a normal: 2 sigma^4 / n
    assert abs(z.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    kurt = np.mean(z ** 4) / z.var() ** 2
    assert abs(kurt - 3.0) < 4.0 * math.sqrt(24.0 / n)
    assert np.max(np.abs(z)) <= omega_bound() + 1e-12
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
