"""Counter-based random streams of the oracle (test infrastructure only).

This module is part of the CPU oracle: plain, slow, obviously correct code
that the tests, the smoke check and the benchmark's CPU baseline use to check
the HIP path.  The product path never imports it.

Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11).  Two independent
implementations live here: a scalar one on Python integers and a vectorised one
on numpy uint64 arrays; the tests check them against each other and against
the generator's published known-answer vectors.

The paper draws its test matrix as ``randn(l, m)`` (Alg. 3, step 2) and takes
its sampling decisions "with probability p" (Alg. 3, prune/fill steps).  Both
draws are realised from Philox streams so that the oracle and the GPU path can
consume the same random numbers; the exact layout is given in
``omega.py`` (test matrix) and ``decision_uniform`` below.
"""
from __future__ import annotations

import numpy as np

# Round multipliers and key increments of Philox4x32 (Salmon et al., SC'11).
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
ROUNDS = 10
MASK32 = 0xFFFFFFFF

# Counter word 3 separates the random streams that may share a seed.
DOMAIN_OMEGA = 0
DOMAIN_DECISION = 1
DOMAIN_DATA = 2

PRUNE_DRAW = 0xFFFFFFFF  # counter word 2 of the prune draw of a slot


def philox4x32_scalar(ctr, key, rounds=ROUNDS):
    """Philox4x32-R on Python ints: ctr is 4 words, key is 2 words."""
    c0, c1, c2, c3 = (int(x) & MASK32 for x in ctr)
    k0, k1 = (int(x) & MASK32 for x in key)
    for rnd in range(rounds):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK32
        hi1, lo1 = p1 >> 32, p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def _mulhilo(a, b):
    """Full 64-bit product of two uint32 arrays, split into (hi, lo) words."""
    p = a.astype(np.uint64) * np.uint64(b)
    return p >> np.uint64(32), p & np.uint64(MASK32)


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Vectorised Philox4x32-R.  Counter words are broadcastable integer
    arrays; the key is two Python ints.  Returns four uint64 arrays holding
    32-bit words."""
    shape = np.broadcast(np.asarray(c0), np.asarray(c1), np.asarray(c2), np.asarray(c3)).shape
    x0 = np.broadcast_to(np.asarray(c0, dtype=np.uint64) & np.uint64(MASK32), shape).copy()
    x1 = np.broadcast_to(np.asarray(c1, dtype=np.uint64) & np.uint64(MASK32), shape).copy()
    x2 = np.broadcast_to(np.asarray(c2, dtype=np.uint64) & np.uint64(MASK32), shape).copy()
    x3 = np.broadcast_to(np.asarray(c3, dtype=np.uint64) & np.uint64(MASK32), shape).copy()
    k0 = int(k0) & MASK32
    k1 = int(k1) & MASK32
    for rnd in range(rounds):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        hi0, lo0 = _mulhilo(x0, PHILOX_M0)
        hi1, lo1 = _mulhilo(x2, PHILOX_M1)
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0)), lo1, (hi0 ^ x3 ^ np.uint64(k1)), lo0
    return x0, x1, x2, x3


def seed_key(seed):
    """Split a 64-bit seed into the two Philox key words (low word first)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & MASK32, seed >> 32


def uniform53(x0, x1):
    """Uniform on [0, 1) with 53 random bits from two 32-bit words; the value
    is exact in binary64: ((x0 >> 5) * 2^26 + (x1 >> 6)) * 2^-53."""
    a = (np.asarray(x0, dtype=np.uint64) >> np.uint64(5)).astype(np.float64)
    b = (np.asarray(x1, dtype=np.uint64) >> np.uint64(6)).astype(np.float64)
    return (a * 67108864.0 + b) * (1.0 / 9007199254740992.0)


def decision_uniform(select_seed, u, i, r):
    """The uniform that decides one Bernoulli draw of the selection step.

    ``u`` is the 0-based update index, ``i`` the basis slot and ``r`` the
    position of the candidate column in the new-column buffer, or
    ``PRUNE_DRAW`` for the prune draw of slot ``i``.  Counter = (u, i, r, 1),
    key = select_seed.  The draw succeeds iff U < p (a draw "with probability
    p", Alg. 3 prune/fill steps)."""
    k0, k1 = seed_key(select_seed)
    x0, x1, _, _ = philox4x32(u, i, r, DOMAIN_DECISION, k0, k1)
    return uniform53(x0, x1)
