"""Whole-stream pins of the oracle (Alg. 3 with Alg. 4) on a small channel
stream: the selection meets the column-subset guarantee of Sec. 2.2.2, and the
ridge parameter does not collapse to its floor once the stream has more
columns than the sketch has rows."""
import math

import numpy as np
import pytest

import synth
from oracle.exact import exact_error, exact_ls
from oracle.rid import Config, OnlineRID


@pytest.fixture(scope="module")
def stream():
    # 4 fields on a 16 x 17 x 16 grid, 600 snapshots (the channel recipe)
    A = synth.channel(16, 17, 16, 600, seed=synth.data_seed(3))
    return np.ascontiguousarray(A.T)


def _run(A, ell, k, t):
    cfg = Config(m=A.shape[0], ell=ell, k=k, t=t, omega_seed=1003, select_seed=2003)
    o = OnlineRID(cfg, n_max=A.shape[1])
    for j0 in range(0, A.shape[1], 100):
        o.push(A[:, j0:j0 + 100])
    o.finalize()
    return o


def test_selection_meets_the_rank_k_guarantee(stream):
    # Sec. 2.2.2: t = O(k log k + k log(1/delta)/eps) columns chosen by ridge
    # leverage scores give ||A - C C^+ A||_F^2 <= (1 + eps) ||A - A_k||_F^2
    # (the guarantee is stated for the rank-k truncation of C C^+ A, whose
    # error is no smaller).  k = 20, t = 100, eps = 0.5.
    A = stream
    o = _run(A, 200, 20, 100)
    Ad = A.astype(np.float64)
    nrm = math.sqrt(float(np.sum(Ad * Ad)))
    sv = np.linalg.svd(Ad, compute_uv=False)
    tail_k = math.sqrt(float(np.sum(sv[20:] ** 2)))
    err_ls = exact_error(A, o.J, exact_ls(A, o.J))
    assert err_ls <= math.sqrt(1.0 + 0.5) * tail_k
    # the one-pass coefficients (Alg. 4) stay within a small factor of that
    err_p = exact_error(A, o.J, o.P)
    assert err_p <= 1.5 * tail_k, (err_p / nrm, tail_k / nrm)


def test_ridge_parameter_leaves_the_floor(stream):
    # k = t = l / 2 as in the paper's runs: once more columns than sketch rows
    # have been seen, the sketch has rank > k and the ridge term is its tail
    o = _run(stream, 200, 100, 100)
    for rec in o.records:
        floor = 1e-8 * rec.F / 100
        if rec.n_obs > 200:
            assert rec.lam > 10.0 * floor, (rec.u, rec.lam, floor)
