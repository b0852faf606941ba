"""Pins of the oracle's sketch S = Omega A (eq. random_sketch; Alg. 3
steps 10-13)."""
import math

import numpy as np

from oracle.omega import omega_entry_scalar, round_to_bf16
from oracle.rid import sketch_columns


def test_brute_force_dense_product():
    rng = np.random.default_rng(1)
    m, ell, b = 37, 11, 5
    A = rng.standard_normal((m, b))
    Om = np.array([[omega_entry_scalar(99, r, i) for i in range(m)] for r in range(ell)])
    S, sq = sketch_columns(A, 99, ell, row_chunk=8)
    expect = np.array([[math.fsum(Om[r, i] * A[i, j] for i in range(m)) for j in range(b)] for r in range(ell)])
    assert np.max(np.abs(S - expect)) <= 1e-13 * np.max(np.abs(expect))
    assert np.allclose(sq, [math.fsum(A[:, j] ** 2) for j in range(b)], rtol=1e-14, atol=0)


def test_linearity():
    rng = np.random.default_rng(2)
    a, b = rng.standard_normal((2, 500))
    Sa, _ = sketch_columns(a[:, None], 3, 17)
    Sb, _ = sketch_columns(b[:, None], 3, 17)
    Sab, _ = sketch_columns((2.5 * a - 0.75 * b)[:, None], 3, 17)
    assert np.allclose(Sab, 2.5 * Sa - 0.75 * Sb, rtol=0, atol=1e-12 * np.abs(Sab).max())


def test_row_chunking_does_not_change_the_sketch():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((1000, 4))
    S1, q1 = sketch_columns(A, 8, 24, row_chunk=1 << 16)
    S2, q2 = sketch_columns(A, 8, 24, row_chunk=77)
    assert np.allclose(S1, S2, rtol=0, atol=1e-12 * np.abs(S1).max())
    assert np.allclose(q1, q2, rtol=1e-14)


def test_expected_sketch_energy():
    # E ||Omega a||^2 = l ||a||^2 for a fixed a and independent unit-variance rows
    rng = np.random.default_rng(4)
    a = rng.standard_normal(256)
    vals = [np.sum(sketch_columns(a[:, None], s, 64)[0] ** 2) for s in range(300)]
    ratio = np.array(vals) / (64 * np.dot(a, a))
    assert abs(ratio.mean() - 1.0) < 4 * ratio.std() / math.sqrt(len(vals))


def test_bf16_operand_form_is_product_of_rounded_operands():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((300, 3)).astype(np.float32)
    S, _ = sketch_columns(A, 6, 16, operand="bf16")
    from oracle.omega import omega_block
    Om = omega_block(6, 16, 0, 300)
    expect = round_to_bf16(Om.astype(np.float32)) @ round_to_bf16(A)
    assert np.allclose(S, expect, rtol=0, atol=1e-12 * np.abs(S).max())
    exact, _ = sketch_columns(A, 6, 16)
    rel = np.linalg.norm(S - exact) / np.linalg.norm(exact)
    assert 1e-4 < rel < 1e-2      # the bf16 rounding is visible and bounded


def test_row_sharded_sketch_sums_to_full():
    # a row-sharded sketch (rows split between devices) is the sum of the
    # shards' sketches, since Omega's counters are global row indices
    rng = np.random.default_rng(6)
    A = rng.standard_normal((900, 3))
    full, fq = sketch_columns(A, 12, 20)
    from oracle.omega import omega_block
    parts = [omega_block(12, 20, r0, r1 - r0) @ A[r0:r1] for r0, r1 in [(0, 250), (250, 700), (700, 900)]]
    assert np.allclose(sum(parts), full, rtol=0, atol=1e-12 * np.abs(full).max())


def test_threaded_chunks_give_the_same_sum():
    # the chunks' products are added in chunk order whatever the thread count
    rng = np.random.default_rng(8)
    A = rng.standard_normal((5000, 7)).astype(np.float32)
    for operand in ("f64", "bf16", "fp8"):
        S1, q1 = sketch_columns(A, 12, 24, operand=operand, row_chunk=512)
        S4, q4 = sketch_columns(A, 12, 24, operand=operand, row_chunk=512, workers=4)
        assert np.array_equal(S1, S4) and np.array_equal(q1, q4)
