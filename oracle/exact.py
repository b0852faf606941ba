"""Exact (multi-pass) reference quantities used by the tests (test
infrastructure only; never imported by the product path).

* ``exact_error``: ||A - A_J P||_F, the quantity Alg. 8 estimates, from a second
  pass over the data (eq. NAhutchPP_expansion, left-hand side).
* ``exact_ls``: P* = A_J^+ A, the least-squares coefficients of eq. coeff_ID2
  (the paper's two-pass "least squares" rows).
"""
from __future__ import annotations

import numpy as np

from .rid import pinv


def exact_error(A, J, P, row_chunk=1 << 16):
    """||A - A_J P||_F in binary64; empty slots (J = -1) contribute nothing."""
    A = np.asarray(A)
    J = np.asarray(J)
    occ = np.flatnonzero(J >= 0)
    tot = 0.0
    for i0 in range(0, A.shape[0], row_chunk):
        blk = A[i0:i0 + row_chunk].astype(np.float64)
        R = blk - blk[:, J[occ]] @ P[occ] if occ.size else blk
        tot += float(np.sum(R * R))
    return float(np.sqrt(tot))


def exact_ls(A, J):
    """P* = A_J^+ A over the occupied slots (rows of empty slots are zero)."""
    A = np.asarray(A, dtype=np.float64)
    J = np.asarray(J)
    P = np.zeros((len(J), A.shape[1]))
    occ = np.flatnonzero(J >= 0)
    if occ.size:
        P[occ] = pinv(A[:, J[occ]]) @ A
    return P
