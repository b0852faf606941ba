"""Pins of the oracle's counter-based generator (Philox4x32-10, Salmon et al.
SC'11) and of the decision uniforms drawn for Alg. 3's prune/fill steps."""
import os

import numpy as np

from oracle.philox import (PRUNE_DRAW, decision_uniform, philox4x32, philox4x32_scalar,
                           seed_key, uniform53)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_kat_scalar():
    for ctr, key, out in _kat():
        assert list(philox4x32_scalar(ctr, key)) == out


def test_kat_vectorised():
    for ctr, key, out in _kat():
        got = philox4x32(*[np.array([c], dtype=np.uint64) for c in ctr], key[0], key[1])
        assert [int(g[0]) for g in got] == out


def test_scalar_matches_vectorised_on_random_inputs():
    rng = np.random.default_rng(123)
    ctr = rng.integers(0, 2**32, (500, 4), dtype=np.uint64)
    for key in [(0, 0), (0xDEADBEEF, 0x12345678), (2**32 - 1, 1)]:
        vec = philox4x32(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], *key)
        for n in range(0, 500, 37):
            assert philox4x32_scalar(ctr[n], key) == tuple(int(v[n]) for v in vec)


def test_seed_key_split():
    assert seed_key(0x0123456789ABCDEF) == (0x89ABCDEF, 0x01234567)


def test_uniform53_range_and_exactness():
    assert uniform53(0, 0) == 0.0
    top = uniform53(0xFFFFFFFF, 0xFFFFFFFF)
    assert top == 1.0 - 2.0 ** -53
    # the 27 + 26 kept bits land exactly: x0 = 1 << 5 is the unit 2^-27
    assert uniform53(1 << 5, 0) == 2.0 ** -27
    assert uniform53(0, 1 << 6) == 2.0 ** -53


def test_decision_uniform_counter_layout():
    k0, k1 = seed_key(77)
    x0, x1, _, _ = philox4x32_scalar((3, 5, PRUNE_DRAW, 1), (k0, k1))
    expect = ((x0 >> 5) * 2.0 ** 26 + (x1 >> 6)) * 2.0 ** -53
    assert float(decision_uniform(77, 3, 5, PRUNE_DRAW)) == expect


def test_decision_uniform_distribution():
    u = decision_uniform(9, np.arange(200000) // 1000, np.arange(200000) % 1000, 0)
    n = u.size
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / n)
    assert abs(np.mean(u < 0.1) - 0.1) < 4 * np.sqrt(0.09 / n)
