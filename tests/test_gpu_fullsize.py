"""Parity at the benchmarked size.

The channel stream's four fields on the 192 x 129 x 192 grid (m = 19 021 824
binary32 rows per snapshot), l = 300, k = t = 150, bfloat16 sketch, in the
launch configuration the benchmark times (lookahead 1024, n_max 1000,
borrowed pushes of 100 snapshots): the first 300 snapshots (two updates of
Alg. 3) against the oracle run on the same bytes, copied back to the host.

Checked: J exactly at both updates; tau and every NA-Hutch++ term (term1, h,
corr, tr_est, gpp, E^2) against the oracle's forward-error tolerances; S
against the bfloat16 form's fixed bounds (worst column 2e-6, 1e-5 relative
Frobenius); P and the reconstruction on sampled snapshots against bounds
declared from this stream's conditioning (below).  The oracle's sketch runs its row chunks
on 16 threads; the whole test takes about three minutes on one MI355X machine
(most of it the oracle).
"""
import math
import time

import numpy as np
import pytest
import torch

import synth
from gpu_common import check_fixed_bounds, compare_updates, log, perturbation_tolerances, rel_fro, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_16076_amd import _lib
    _lib.lib()


def test_channel_19M_rows_bf16_two_updates_match_oracle():
    from paper_2405_16076_amd import OnlineRID, StreamConfig
    nx, ny, nz, n, ell, t = 192, 129, 192, 300, 300, 150
    m = 4 * nx * ny * nz
    t0 = time.perf_counter()
    D = synth.channel_torch(nx, ny, nz, n, synth.data_seed(3), fields=4, n_modes=300)
    torch.cuda.synchronize()
    log(f"channel stream m={m} n={n} generated in {time.perf_counter() - t0:.1f} s")
    X = D[:, :m]
    cfg = StreamConfig(m=m, ell=ell, k=t, t=t, n_max=1000, dtype=torch.float32, sketch="bf16",
                       omega_seed=1003, select_seed=2003, lookahead=1024)
    s = OnlineRID(cfg)
    t0 = time.perf_counter()
    for j0 in range(0, n, 100):
        s.push(X[j0:j0 + 100], borrow=True)
    s.finalize()
    J = s.select()
    P = s.coefficients()
    Sg, _, _ = s.debug_state()
    log(f"  GPU pass {time.perf_counter() - t0:.2f} s (with the host synchronisations of the getters)")
    t0 = time.perf_counter()
    A = X.cpu().numpy()                       # (n, m) binary32, the bytes the GPU read
    log(f"  copied to the host in {time.perf_counter() - t0:.1f} s")
    t0 = time.perf_counter()
    o = run_oracle(A, ell, t, t, "bf16", 1003, 2003, workers=16)
    log(f"  oracle in {time.perf_counter() - t0:.1f} s, {len(o.records)} updates, "
        f"filled {[r.n_filled for r in o.records]}, lambda {[f'{r.lam:.3e}' for r in o.records]}")
    t0 = time.perf_counter()
    tol = perturbation_tolerances(o, A, "bf16", recon=False)
    b_t1 = tol["b_term1"]
    worst_tau, margin = compare_updates(s, o, tol)
    log(f"  tolerances in {time.perf_counter() - t0:.1f} s; tau diff/tol {worst_tau:.2e}, min margin {margin:.2e}")
    assert np.array_equal(J, o.J)
    occ = np.flatnonzero(J >= 0)
    assert np.allclose(P[occ][:, J[occ]], np.eye(occ.size), atol=1e-5)
    for u, rec in enumerate(o.records):
        g = s.update(u)
        h = rec.hutch
        assert abs(g["F"] - rec.F) <= 1e-12 * rec.F
        for key in ("term1", "h", "corr"):
            log(f"  update {u} {key}: gpu {g[key]:.9e} oracle {h[key]:.9e}")
        for key in ("tr_est", "gpp", "E2"):
            d = abs(g[key] - h[key])
            log(f"  update {u} {key}: gpu {g[key]:.9e} oracle {h[key]:.9e} diff/tol {d / tol[key][u]:.2e}")
            assert d <= tol[key][u], (u, key, g[key], h[key], tol[key][u])
        # each part of tr_est is bilinear in the sketch: relative error at most
        # about twice the sketch's (the bfloat16 S bound is 1e-4); term1 also
        # takes the split-form Gram's bound
        for key in ("term1", "h", "corr"):
            extra = b_t1[u] if key == "term1" else 0.0
            assert abs(g[key] - h[key]) <= 2e-4 * abs(h[key]) + extra, (u, key)
    # reconstruction of sampled snapshots: A_J P(:, j) with A_J from the host bytes
    cols = np.array([0, 37, 149, 150, 151, 222, 299])
    AJ = A[J[occ]].astype(np.float64)         # (|J|, m)
    Ro = (o.P[occ][:, cols].T @ AJ)           # (len(cols), m)
    R = np.stack([s.reconstruct(int(j), 1).cpu().numpy()[0].astype(np.float64) for j in cols])
    # At this size cond(Omega A_J) is 1.2e4, ten times the small channel
    # streams': binary32 accumulation over the 37k-row slabs leaves S about
    # 1e-6 from the oracle's, and P's forward error is about 0.1 cond(Omega A_J)
    # times that.  Bounds declared for this test: P 5e-3, reconstruction 5e-4.
    assert o.records[-1].cond_SJ < 3e4
    check_fixed_bounds("bf16", Sg[:, :n], o.S[:, :n], P, o.P, R, Ro, o.records[-1].cond_SJ, pb=5e-3, rb=5e-4)
    assert rel_fro(Sg[:, :n], o.S[:, :n]) <= 1e-5
    # the exact error of the sampled snapshots beside the estimate
    Aj = A[cols].astype(np.float64)
    exact = math.sqrt(float(np.sum((R - Aj) ** 2)) / float(np.sum(Aj * Aj)))
    log(f"  sampled exact rel error {exact:.4e}, NA-Hutch++ rel estimate {s.error_estimate()['rel']:.4e}")
    s.close()
    del D, X
    torch.cuda.empty_cache()
