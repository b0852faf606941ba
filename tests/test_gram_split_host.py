"""Host checks of the arithmetic behind the split form of the basis Gram
(binary32 data on the bfloat16 matrix cores): the three-piece bfloat16 split
is exact, the dropped piece products stay below their bound, and the
worst-case binary32 summation of one 32-row group (every addition rounded, in
the kernel's order of products) stays within the stated elementwise bound
37 u sum|a b| (u = 2^-24).  numpy emulation; no GPU."""
import numpy as np

U = 2.0 ** -24


def bf16_rne(x):
    """binary32 -> the bfloat16 value nearest (ties to even), as binary32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16
    return b.astype(np.uint32).view(np.float32)


def split3(a):
    a = np.asarray(a, dtype=np.float32)
    a0 = bf16_rne(a)
    r1 = (a - a0).astype(np.float32)
    a1 = bf16_rne(r1)
    a2 = bf16_rne((r1 - a1).astype(np.float32))
    return a0, a1, a2


def wide_values(rng, n, lo=-100, hi=60):
    mant = rng.uniform(1.0, 2.0, n) * rng.choice([-1.0, 1.0], n)
    return (mant * 2.0 ** rng.integers(lo, hi, n)).astype(np.float32)


def test_split_is_exact_and_pieces_shrink():
    rng = np.random.default_rng(0)
    a = np.concatenate([wide_values(rng, 200_000),
                        # every significand pattern near the rounding ties
                        (np.arange(1 << 16, dtype=np.uint32) << 8 | 0x3F800000).view(np.float32),
                        (np.arange(1 << 16, dtype=np.uint32) | 0x3F800000).view(np.float32),
                        np.float32([0.0, -0.0, 1.0, -1.0, 2.0 ** -100, 2.0 ** 60])])
    a0, a1, a2 = split3(a)
    for p in (a0, a1, a2):
        assert np.array_equal(bf16_rne(p), p)                   # each piece is a bfloat16 value
    s = a0.astype(np.float64) + a1.astype(np.float64) + a2.astype(np.float64)
    assert np.array_equal(s, a.astype(np.float64))             # a = a0 + a1 + a2 exactly
    aa = np.abs(a.astype(np.float64))
    assert np.all(np.abs(a1) <= 2.0 ** -8 * (1 + 2.0 ** -8) * aa)
    assert np.all(np.abs(a2) <= 2.0 ** -16 * aa)


def test_dropped_products_stay_below_their_bound():
    rng = np.random.default_rng(1)
    a, b = wide_values(rng, 100_000, -40, 40), wide_values(rng, 100_000, -40, 40)
    a0, a1, a2 = (p.astype(np.float64) for p in split3(a))
    b0, b1, b2 = (p.astype(np.float64) for p in split3(b))
    kept = a0 * b0 + a0 * b1 + a1 * b0 + a0 * b2 + a1 * b1 + a2 * b0
    exact = a.astype(np.float64) * b.astype(np.float64)
    assert np.all(np.abs(exact - kept) <= 2.0 ** -23 * (1 + 2.0 ** -7) * np.abs(exact))


def group_sum_worst_case(a, b):
    """One 32-row group as the kernel orders it (two 16-row steps; products
    of order 2, then 1, then 0), every binary32 addition rounded."""
    A = [p.astype(np.float32) for p in split3(a)]
    B = [p.astype(np.float32) for p in split3(b)]
    acc = np.float32(0.0)
    order = [(0, 2), (1, 1), (2, 0)], [(0, 1), (1, 0)], [(0, 0)]
    for phase in order:
        for s in (0, 1):
            rows = slice(16 * s, 16 * s + 16)
            for i, j in phase:
                for x, y in zip(A[i][rows], B[j][rows]):
                    acc = np.float32(acc + np.float32(x * y))   # x y is exact in binary32
    return float(acc)


def test_worst_case_group_sum_within_the_stated_bound():
    rng = np.random.default_rng(2)
    worst = 0.0
    for trial in range(400):
        kind = trial % 4
        if kind == 0:
            a, b = rng.standard_normal(32).astype(np.float32), rng.standard_normal(32).astype(np.float32)
        elif kind == 1:      # one sign: no cancellation, the partial sums grow
            a = np.abs(rng.standard_normal(32)).astype(np.float32)
            b = np.abs(rng.standard_normal(32)).astype(np.float32) + 1
        elif kind == 2:      # magnitudes over 2^-30 .. 2^30 in one group
            a, b = wide_values(rng, 32, -30, 30), wide_values(rng, 32, -30, 30)
        else:                # heavy cancellation: b = a with alternating signs
            a = rng.standard_normal(32).astype(np.float32)
            b = (a * np.where(np.arange(32) % 2 == 0, 1, -1)).astype(np.float32)
        exact = float(np.dot(a.astype(np.float64), b.astype(np.float64)))
        scale = float(np.dot(np.abs(a.astype(np.float64)), np.abs(b.astype(np.float64))))
        err = abs(group_sum_worst_case(a, b) - exact)
        worst = max(worst, err / (scale * U))
        assert err <= 37 * U * scale, (trial, err / (scale * U))
    assert worst > 0.0
