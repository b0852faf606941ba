"""Pins of the oracle's e4m3 operands (the fp8 sketch form).

The reference here is independent of the oracle's arithmetic: the 256 e4m3
codes are decoded from their bit fields (1 sign, 4 exponent with bias 7,
3 mantissa bits; exponent 0 subnormal; 0x7F / 0xFF not finite), and rounding
is an exhaustive nearest-code search with ties to the code of even mantissa,
saturating at the largest finite magnitude (OCP 8-bit floating point
specification, e4m3)."""
import math

import numpy as np

import oracle
from oracle.omega import (E4M3_MAX, mx_block_exponent, quantize_fp8_blocks, quantize_fp8_omega,
                          round_to_e4m3)


def _decode(code):
    s, e, m = code >> 7, (code >> 3) & 15, code & 7
    if e == 15 and m == 7:
        return None
    v = (m / 8.0) * 2.0 ** -6 if e == 0 else (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return -v if s else v


_CODES = [(c, _decode(c)) for c in range(256) if _decode(c) is not None]


def _nearest(x):
    if abs(x) >= E4M3_MAX:
        return math.copysign(E4M3_MAX, x)
    best = None
    for c, v in _CODES:
        d = abs(v - x)
        if best is None or d < best[0] or (d == best[0] and (c & 1) == 0 and (best[1] & 1) == 1):
            best = (d, c, v)
    return best[2]


def test_every_code_round_trips():
    vals = np.array([v for _, v in _CODES])
    assert np.array_equal(round_to_e4m3(vals), vals)
    assert max(abs(v) for v in vals) == 448.0 and len(set(vals)) == 253  # +-0 equal


def test_midpoints_round_to_even_and_saturate():
    pos = sorted(set(abs(v) for _, v in _CODES))
    mids = [(a + b) / 2 for a, b in zip(pos[:-1], pos[1:])]
    xs = np.array(mids + [-m for m in mids] + [448.0, 460.0, 463.99, 464.0, 500.0, 1e6, -1e6, 2 ** -10, 3 * 2 ** -10])
    want = np.array([_nearest(float(x)) for x in xs])
    assert np.array_equal(round_to_e4m3(xs), want)


def test_random_values_match_exhaustive_search():
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.standard_normal(3000) * 10.0 ** rng.uniform(-4, 3, 3000),
                         rng.uniform(-470, 470, 500)])
    want = np.array([_nearest(float(x)) for x in xs])
    assert np.array_equal(round_to_e4m3(xs), want)


def test_block_scale_puts_the_maximum_in_range():
    rng = np.random.default_rng(4)
    for _ in range(200):
        amax = 10.0 ** rng.uniform(-30, 30)
        e = int(mx_block_exponent(amax))
        assert 128.0 <= amax / 2.0 ** e < 256.0
    assert int(mx_block_exponent(0.0)) == -127


def test_block_quantization_error_and_alignment():
    rng = np.random.default_rng(5)
    # columns with a wide dynamic range across blocks of 32 rows
    x = rng.standard_normal((96, 5)) * 10.0 ** rng.uniform(-6, 6, (3, 1)).repeat(32, axis=0)
    q = quantize_fp8_blocks(x)
    for r0 in range(0, 96, 32):
        part, qp = x[r0:r0 + 32], q[r0:r0 + 32]
        amax = np.max(np.abs(part), axis=0)
        e = np.floor(np.log2(amax)) - 7
        sc = 2.0 ** e
        # every element is one of the grid values of its block
        for j in range(5):
            for i in range(32):
                assert qp[i, j] == _nearest(part[i, j] / sc[j]) * sc[j]
    # error bound: half a unit of the last place of e4m3 in normal range,
    # 2^-10 of the scale below it
    rel_ok = np.abs(q - x) <= np.maximum(np.abs(x) * 2.0 ** -4, 2.0 ** -10 * np.repeat(
        2.0 ** (np.floor(np.log2(np.max(np.abs(x).reshape(3, 32, 5), axis=1))) - 7), 32, axis=0))
    assert rel_ok.all()


def test_omega_operand_is_the_scaled_grid():
    om = oracle.omega_block(9, 24, 0, 200)
    q = quantize_fp8_omega(om)
    want = np.array([[_nearest(float(v) * 64.0) / 64.0 for v in row] for row in om])
    assert np.array_equal(q, want)
    assert np.max(np.abs(om)) * 64.0 < 448.0  # Omega is bounded by 4.7098: no saturation


def test_fp8_sketch_is_the_product_of_quantized_operands():
    rng = np.random.default_rng(6)
    m, b, ell = 200, 4, 12
    A = (rng.standard_normal((m, b)) * np.array([1e-3, 1.0, 1e3, 1e5])).astype(np.float32)
    S, _ = oracle.sketch_columns(A, 17, ell, operand="fp8", row_chunk=64)
    om = oracle.omega_block(17, ell, 0, m)
    Oq = np.array([[_nearest(float(v) * 64.0) / 64.0 for v in row] for row in om])
    Aq = np.zeros((m, b))
    for r0 in range(0, m, 32):
        part = A[r0:r0 + 32].astype(np.float64)
        sc = 2.0 ** (np.floor(np.log2(np.max(np.abs(part), axis=0))) - 7)
        Aq[r0:r0 + 32] = np.array([[_nearest(part[i, j] / sc[j]) * sc[j] for j in range(b)] for i in range(part.shape[0])])
    assert np.allclose(S, Oq @ Aq, rtol=1e-13, atol=0)
    # and it stays close to the exact sketch (e4m3 has 3 mantissa bits)
    Sx, _ = oracle.sketch_columns(A, 17, ell, operand="f64")
    assert np.linalg.norm(S - Sx) / np.linalg.norm(Sx) < 0.1
