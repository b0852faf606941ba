"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances:
* Omega: the binary32, bfloat16 and e4m3 forms equal the oracle's rounding of
  the same binary64 table entry bit for bit; the binary64 form is within a
  few ulp (the two sides compute the quantiles with different algorithms).
* Sketch S: binary64 sums in another order (1e-12 relative Frobenius);
  binary32 accumulation within a row slab (2e-5); bfloat16 against the
  oracle's product of the same bfloat16 operands (1e-5: binary32 accumulation
  only); fp8 against the oracle's product of the same e4m3 codes and block
  scales (1e-3: the scaled MFMA rounds inside each 64-term product).
* Coefficients P, the reconstruction A_J P and the worst column of S are held
  to fixed bounds declared per form in gpu_common (P_BOUND, RECON_BOUND,
  S_COL_BOUND): binary64 1e-10; binary32 1e-5 (P only where cond(Omega A_J)
  <= 100, else 1e-3, with the reconstruction still at 1e-5); bfloat16 P 1e-3,
  reconstruction 1e-4; e4m3 P 3e-3, reconstruction 1e-3.
* The scores tau and the NA-Hutch++ terms are compared with a forward-error
  tolerance computed by the oracle itself: its own S is perturbed at the
  sketch accuracy of the form and the step is recomputed; the tolerance is 10x
  the largest change seen (gpu_common.perturbation_tolerances); the same
  derived tolerance of P is logged beside its fixed bound.  The index sets J
  must match exactly (the smallest decision margin |U - p| is logged).
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import (check_fixed_bounds, compare_updates, gram_split_eps, log, perturbation_tolerances, rel_fro,
                        run_gpu, run_oracle, split_gram_bounds, uses_gram_split)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_16076_amd import _lib
    _lib.lib()


# ---------------------------------------------------------------------------
# Omega
# ---------------------------------------------------------------------------
def test_omega_f64_matches_oracle():
    # both sides hold binary64 quantiles of the same definition, computed by
    # different algorithms: a few ulp apart
    from paper_2405_16076_amd import omega_block
    for seed, ell, i0, cnt in [(1001, 40, 0, 5000), (7, 301, (1 << 32) - 100, 300)]:
        log("omega f64", seed, ell, i0, cnt)
        g = omega_block("f64", seed, ell, i0, cnt).cpu().numpy()
        o = oracle.omega_block(seed, ell, i0, cnt)
        assert np.max(np.abs(g - o)) <= 8 * np.finfo(np.float64).eps * np.max(np.abs(o))
        assert np.array_equal(np.sign(g), np.sign(o))


def test_omega_f32_bf16_fp8_equal_the_oracle_bit_for_bit():
    # every reduced-precision form holds the rounding of the same table entry
    from paper_2405_16076_amd import omega_block
    seed, ell, cnt = 2024, 320, 20000
    o = oracle.omega_block(seed, ell, 0, cnt)
    g = omega_block("f32", seed, ell, 0, cnt).cpu().numpy().astype(np.float64)
    assert np.array_equal(g, o.astype(np.float32).astype(np.float64))
    gb = omega_block("bf16", seed, ell, 0, cnt).cpu().numpy().astype(np.float64)
    assert np.array_equal(gb, oracle.round_to_bf16(o))
    g8 = omega_block("fp8", seed, ell, (1 << 32) - 7, cnt).cpu().numpy().astype(np.float64)
    assert np.array_equal(g8, oracle.quantize_fp8_omega(oracle.omega_block(seed, ell, (1 << 32) - 7, cnt)))


# ---------------------------------------------------------------------------
# sketch S = Omega A and ||a_j||^2
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("sketch,m,n,ell,tol,tile", [
    ("f64", 4096, 64, 40, 1e-12, "auto"),
    ("f64", 3001, 33, 71, 1e-12, "auto"),
    ("f32", 100_003, 300, 40, 2e-5, "auto"),
    ("f32", 70_000, 70, 300, 2e-5, "auto"),
    ("bf16", 100_003, 300, 40, 1e-5, "auto"),
    # l = 300: the wide tile (two workgroups per 512 columns) and the narrow one
    ("bf16", 65_536, 600, 300, 1e-5, "auto"),
    ("bf16", 65_536, 600, 300, 1e-5, "wide"),
    # wide tile with 3 and 4 row blocks per workgroup, ragged rows and columns
    ("bf16", 40_009, 530, 150, 1e-5, "wide"),
    ("bf16", 33_333, 1030, 200, 1e-5, "wide"),
    # fp8: same e4m3 codes and scales as the oracle; the scaled MFMA rounds
    # inside each 64-term product (~1e-4 of S, see SKETCH_ACCURACY)
    ("fp8", 100_003, 300, 40, 1e-3, "auto"),
    ("fp8", 65_536, 600, 300, 1e-3, "auto"),
])
def test_sketch_matches_oracle(sketch, m, n, ell, tol, tile):
    log("sketch", sketch, m, n, ell, tile)
    rng = np.random.default_rng(m + n)
    dt = np.float64 if sketch == "f64" else np.float32
    A = rng.standard_normal((n, m)).astype(dt)
    s = run_gpu(A, ell, k=4, t=4, sketch=sketch, omega_seed=77, select_seed=78, finalize=False, lookahead=256,
                tile=tile)
    S, q, _ = s.debug_state()
    So, qo = oracle.sketch_columns(A.T, 77, ell, operand=sketch)
    e = rel_fro(S, So)
    log("  rel fro", e, "colsq max rel", np.max(np.abs(q - qo) / qo))
    assert e <= tol
    assert np.max(np.abs(q - qo) / qo) <= 1e-13


@pytest.mark.parametrize("sketch,ell,tile", [("f32", 64, "auto"), ("bf16", 64, "auto"), ("bf16", 300, "auto"),
                                             ("bf16", 300, "wide"), ("fp8", 300, "auto")])
def test_sketch_is_independent_of_batching(sketch, ell, tile):
    log("batching independence", sketch, ell, tile)
    rng = np.random.default_rng(5)
    A = rng.standard_normal((200, 50_001)).astype(np.float32)
    ref = run_gpu(A, ell, 8, 8, sketch, 3, 4, finalize=False, lookahead=256, tile=tile).debug_state()
    for batch, la in [(1, 0), (7, 100), (64, 64)]:
        got = run_gpu(A, ell, 8, 8, sketch, 3, 4, batch=batch, finalize=False, lookahead=la,
                      tile=tile).debug_state()
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("sketch", ["f32", "bf16"])
def test_pipeline_is_independent_of_batching(sketch):
    """SS^T of update u is SS^T of update u - 1 plus the products of update
    u's own columns, so the scores, the selection, P and every NA-Hutch++ term
    are bitwise the same however the pushes fall into flushes."""
    log("pipeline batching independence", sketch)
    A = synth.lowrank(20_011, 260, seed=11, rank=40, rel_noise=1e-3)
    runs = []
    for batch, la in [(None, 0), (7, 30), (64, 64), (130, 256)]:
        s = run_gpu(A, 40, 20, 20, sketch, 21, 22, batch=batch, lookahead=la)
        recs = [s.update(u) for u in range(int(s.info().n_updates))]
        runs.append((s.select(), s.coefficients(), recs, (batch, la)))
    J0, P0, R0, _ = runs[0]
    for J, P, R, how in runs[1:]:
        assert np.array_equal(J, J0), how
        assert np.array_equal(P, P0), how
        assert len(R) == len(R0)
        for a, b in zip(R, R0):
            for key in ("F", "sk2", "lam", "E2", "tr_est", "gpp"):
                assert a[key] == b[key], (how, a["update"], key, a[key], b[key])
            assert np.array_equal(a["J"], b["J"]) and np.array_equal(a["tau_C"], b["tau_C"], equal_nan=True)


# ---------------------------------------------------------------------------
# whole stream: J, tau, P, E^2, reconstruction
# ---------------------------------------------------------------------------
def _pipeline(A, ell, k, t, sketch, oseed, sseed, batch=None, borrow=True, n_max=None, lookahead=0):
    s = run_gpu(A, ell, k, t, sketch, oseed, sseed, batch=batch, borrow=borrow, n_max=n_max, lookahead=lookahead)
    o = run_oracle(A, ell, k, t, sketch, oseed, sseed)
    tol = perturbation_tolerances(o, A, sketch)
    worst_tau, margin = compare_updates(s, o, tol)
    log(f"  updates {len(o.records)} tau diff/tol {worst_tau:.2e} min margin {margin:.2e} "
        f"max kappa {max(r.kappa for r in o.records if r.tau_D is not None):.2e}")
    J = s.select()
    assert np.array_equal(J, o.J)
    P = s.coefficients()
    occ = J >= 0
    assert np.allclose(P[occ][:, J[occ]], np.eye(int(occ.sum())), atol=1e-9 if sketch == "f64" else 1e-5)
    # NA-Hutch++ terms of every update
    worst = {}
    for u, rec in enumerate(o.records):
        g = s.update(u)
        h = rec.hutch
        assert abs(g["F"] - rec.F) <= 1e-12 * max(rec.F, 1e-300)
        for key in ("tr_est", "gpp", "E2"):
            d = abs(g[key] - h[key])
            worst[key] = max(worst.get(key, 0.0), d / tol[key][u])
            assert d <= tol[key][u], (u, key, g[key], h[key], tol[key][u])
    log("  NA-Hutch++ diff/tol " + " ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    Sg, _, G = s.debug_state()
    # the last update's ||S_k||^2 and lambda' (tridiagonalisation, multisection
    # and ridge kernels) against LAPACK's eigenvalues of the device's own S S^T
    last = s.update(len(o.records) - 1)
    Sd = Sg[:, :o.n_obs].astype(np.float64)
    SST = Sd @ Sd.T
    tr = float(np.trace(SST))
    sk2 = float(np.sum(np.linalg.eigvalsh(SST)[::-1][:min(k, ell)]))
    assert abs(last["sk2"] - sk2) <= 1e-10 * tr, (last["sk2"], sk2, tr)
    lam = max(last["F"] * (tr - last["sk2"]) / tr / k, 1e-8 * last["F"] / k)
    assert abs(last["lam"] - lam) <= 1e-8 * lam + 1e-12 * last["F"] / k, (last["lam"], lam)
    eg = rel_fro(G, o.G)
    log(f"  Gram rel fro {eg:.2e}")
    if uses_gram_split(sketch):
        # the split form's bound, through sum_r |a_ri||a_rj| <= sqrt(G_ii G_jj)
        dgo = np.sqrt(np.abs(np.diag(o.G)))
        assert np.all(np.abs(G - o.G) <= gram_split_eps(A.shape[1]) * np.outer(dgo, dgo))
    else:
        assert eg <= 1e-12
    # S, P and the reconstruction of a column range against fixed bounds
    n = A.shape[0]
    c0, c = max(0, n // 2 - 5), min(17, n)
    R = s.reconstruct(c0, c).cpu().numpy().astype(np.float64)
    occi = np.flatnonzero(occ)
    Ro = (A.T[:, J[occi]].astype(np.float64) @ o.P[occi][:, c0:c0 + c]).T
    check_fixed_bounds(sketch, Sg[:, :o.n_obs], o.S[:, :o.n_obs], P, o.P, R, Ro, o.records[-1].cond_SJ, tol)
    return s, o


def test_pipeline_f64_sines():
    log("pipeline f64 sines 4096 x 512, l=40, t=20")
    A = synth.sines(4096, 512, seed=synth.data_seed(1))
    _pipeline(A, 40, 20, 20, "f64", 1001, 2001)


def test_pipeline_f64_ragged_small_batches_copy():
    log("pipeline f64 ragged, copy pushes of 7")
    A = synth.sines(1000, 97, seed=3)
    _pipeline(A, 24, 8, 8, "f64", 5, 6, batch=7, borrow=False)


def test_pipeline_f32_lowrank():
    log("pipeline f32 lowrank 65536 x 400, l=40, t=20")
    A = synth.lowrank(65536, 400, seed=synth.data_seed(2), rank=60)
    _pipeline(A, 40, 20, 20, "f32", 1002, 2002, batch=32)


def test_pipeline_f32_channel():
    log("pipeline f32 channel 24x17x24x4, l=60, t=30")
    A = synth.channel(24, 17, 24, 300, seed=synth.data_seed(3), n_modes=120)
    _pipeline(A, 60, 30, 30, "f32", 1003, 2003)


def test_pipeline_f32_lowrank_large_ell():
    # l = 300, t = 150 as in the full-size channel workload (register-resident
    # QR, NA-Hutch++ split 75/150/75), on a well-conditioned stream: the
    # spectrum decays slowly, so Omega A_J is far from rank-deficient.
    log("pipeline f32 lowrank 40000 x 450, rank 400, l=300, t=150")
    A = synth.lowrank(40_000, 450, seed=synth.data_seed(2), rank=400, decay=200.0)
    _pipeline(A, 300, 150, 150, "f32", 1003, 2003, batch=100)


def test_pipeline_f32_lowrank_ell400_fallback_kernels():
    # l = 400, t = 200 (the sizes of the ignition configuration): seven
    # elements per lane in the tridiagonalisation, Alg. 4 through the L2
    # QR and the per-column solve (t > 154), NA-Hutch++ through the L2 kernel
    log("pipeline f32 lowrank 8192 x 500, rank 450, l=400, t=200")
    A = synth.lowrank(8192, 500, seed=synth.data_seed(5), rank=450, decay=300.0)
    _pipeline(A, 400, 200, 200, "f32", 1005, 2005, batch=100)


def test_pipeline_f32_ell400_coefficients_one_update_at_a_time():
    # n_max so large that one update's P (t x n_max, 640 MB) passes the cap on
    # the per-update P slices: the Alg. 4 / Alg. 8 phases of the flush's three
    # updates run one update at a time on the second stream
    log("pipeline f32 lowrank 8192 x 500, l=400, t=200, n_max=400000, one flush")
    A = synth.lowrank(8192, 500, seed=synth.data_seed(5), rank=450, decay=300.0)
    _pipeline(A, 400, 200, 200, "f32", 1005, 2005, n_max=400_000, lookahead=1024)


def test_pipeline_bf16_channel_operand_rounding():
    log("pipeline bf16 channel vs oracle with bf16-rounded operands")
    A = synth.channel(24, 17, 24, 300, seed=synth.data_seed(3), n_modes=120)
    _pipeline(A, 60, 30, 30, "bf16", 1003, 2003)


def test_pipeline_fp8_channel_operand_rounding():
    log("pipeline fp8 channel vs oracle with e4m3 operands")
    A = synth.channel(24, 17, 24, 300, seed=synth.data_seed(3), n_modes=120)
    _pipeline(A, 60, 30, 30, "fp8", 1003, 2003)


def test_fewer_columns_than_slots_gives_zero_error():
    log("n < t: one partial update keeps every column")
    rng = np.random.default_rng(9)
    A = rng.standard_normal((6, 5000))
    s = run_gpu(A, 32, 8, 8, "f64", 3, 4)
    J = s.select()
    assert sorted(J[J >= 0]) == list(range(6))
    R = s.reconstruct(0, 6).cpu().numpy()
    assert rel_fro(R, A) <= 1e-12
    assert abs(s.error_estimate()["E2"]) <= 1e-9 * float(np.sum(A * A))


def test_zero_stream_skips_selection():
    A = np.zeros((10, 777))
    s = run_gpu(A, 16, 4, 4, "f64", 1, 2)
    rec = s.update(0)
    from paper_2405_16076_amd import _lib
    assert rec["flags"] & _lib.RID_UPD_SKIPPED
    assert np.all(s.select() == -1)
    assert s.error_estimate()["E2"] == 0.0


def test_non_finite_input_latches_enumeric():
    from paper_2405_16076_amd import RIDError
    A = np.ones((8, 1000), dtype=np.float32)
    A[3, 17] = np.nan
    s = run_gpu(A, 16, 4, 4, "f32", 1, 2, finalize=False)
    with pytest.raises(RIDError) as ei:
        s.select()
    assert ei.value.status == 6
    info = s.info()
    assert info.failed == 1


def test_reset_and_rerun_are_bitwise_identical():
    A = synth.lowrank(20000, 120, seed=11, rank=30)
    s = run_gpu(A, 32, 10, 10, "f32", 8, 9, batch=40)
    J1, P1 = s.select(), s.coefficients()
    s.reset()
    X = s._data
    for j0 in range(0, 120, 25):
        s.push(X[j0:j0 + 25], borrow=False)
    s.finalize()
    assert np.array_equal(s.select(), J1)
    assert np.array_equal(s.coefficients(), P1)


def test_back_to_back_passes_without_host_sync():
    # rid_reset does not wait for the device: passes over two streams are
    # enqueued one after another (copied and borrowed columns, the pinned
    # column table rewritten each time) and the last one must equal a fresh run
    A = synth.lowrank(20000, 120, seed=11, rank=30)
    B = synth.lowrank(20000, 120, seed=12, rank=40)
    sb = run_gpu(B, 32, 10, 10, "f32", 8, 9, batch=40)
    JB, PB = sb.select(), sb.coefficients()
    s = run_gpu(A, 32, 10, 10, "f32", 8, 9, batch=40)
    XA, XB = s._data, sb._data
    for X, borrow in ((XB, False), (XA, True), (XB, True), (XA, False), (XB, True)):
        s.reset()
        for j0 in range(0, 120, 25):
            s.push(X[j0:j0 + 25], borrow=borrow)
        s.finalize()
    assert np.array_equal(s.select(), JB)
    assert np.array_equal(s.coefficients(), PB)


def _gram_check(G, A_cols, J, gram, m, label=""):
    """G against A_J^T A_J from the host bytes: binary64 products within 1e-13
    of sqrt(G_ii G_jj); the split form within its stated bound
    eps(m) sum_r |a_ri| |a_rj| elementwise.  Returns the worst ratio to the bound."""
    t = J.size
    occ = np.flatnonzero(J >= 0)
    X = A_cols[J[occ]].astype(np.float64)
    Gx = np.zeros((t, t))
    Gx[np.ix_(occ, occ)] = X @ X.T
    if gram == "split":
        Ga = np.zeros((t, t))
        Ga[np.ix_(occ, occ)] = np.abs(X) @ np.abs(X).T
        bound = gram_split_eps(m) * Ga
    else:
        bound = 1e-13 * np.sqrt(np.outer(np.diag(Gx), np.diag(Gx)))
    err = np.abs(G - Gx)
    ratio = np.where(bound > 0, err / np.where(bound > 0, bound, 1.0), np.where(err > 0, np.inf, 0.0))
    scaled = err / np.sqrt(np.outer(np.diag(Gx), np.diag(Gx)) + 1e-300)
    log(f"  {label}Gram ({gram}) max scaled err {scaled.max():.2e}, worst err/bound {ratio.max():.2e}")
    assert ratio.max() <= 1.0, (gram, float(ratio.max()))
    return float(ratio.max())


@pytest.mark.parametrize("dtype,gram", [(np.float64, "auto"), (np.float32, "exact"), (np.float32, "split")])
def test_gram_and_estimate_terms_after_first_update(dtype, gram):
    # G = A_J^T A_J: binary64 products (exact for binary32 data), or the split
    # form within its bound; each NA-Hutch++ term is checked against the oracle
    # separately (well-conditioned data); gpp also takes the split form's bound
    rng = np.random.default_rng(21)
    m, t, ell = 4099, 40, 80
    A = (rng.standard_normal((t, 12)) @ rng.standard_normal((12, m)) + 0.1 * rng.standard_normal((t, m))).astype(dtype)
    sk = "f64" if dtype == np.float64 else "f32"
    s = run_gpu(A, ell, t, t, sk, 31, 32, gram=gram)
    o = run_oracle(A, ell, t, t, sk, 31, 32)
    _, _, G = s.debug_state()
    J = s.select()
    occ = np.flatnonzero(J >= 0)
    _gram_check(G, A, J, "split" if gram == "split" else "exact", m)
    g = s.update(0)
    h = o.records[0].hutch
    log("  terms gpu " + " ".join(f"{k}={g[k]:.6e}" for k in ("term1", "h", "corr", "gpp", "E2")))
    log("  terms orc " + " ".join(f"{k}={h[k]:.6e}" for k in ("term1", "h", "corr", "gpp", "E2")))
    extra = {}
    if gram == "split":  # n = t: one update, o.P is its P
        SJ = np.zeros((ell, t))
        SJ[:, occ] = o.S[:, J[occ]]
        extra["term1"], extra["gpp"] = split_gram_bounds(o.S[:, :A.shape[0]], SJ, o.P, G, o.cfg.n1, o.cfg.n2, m, occ)
    for k in ("term1", "h", "corr", "gpp"):
        assert abs(g[k] - h[k]) <= 1e-7 * max(abs(h[k]), o.F) + extra.get(k, 0.0), k


@pytest.mark.parametrize("dtype,m,t,growth,gram", [(np.float32, 20_011, 150, 1.02, "split"),
                                                   (np.float32, 20_011, 150, 1.02, "exact"),
                                                   (np.float32, 9_001, 100, 1.0, "split"),
                                                   (np.float32, 9_001, 100, 1.0, "exact"),
                                                   (np.float32, 12_007, 200, 1.0, "split"),
                                                   (np.float32, 10_007, 60, "dyn", "split"),
                                                   (np.float64, 8_011, 100, 1.0, "auto")])
def test_gram_after_every_update(dtype, m, t, growth, gram):
    # after each update G must equal A_J^T A_J of that update's J (binary64
    # products: to 1e-13; split form: within its stated bound); partial refills
    # of varied size exercise the new-by-new blocks taken from their mirrors
    # and the blocks past the ends of the lists; t = 200 (224 staged columns)
    # takes the single-buffered split planes; "dyn" draws magnitudes over 2^-40 .. 2^40
    # inside every column (the split is exact at any exponent)
    from paper_2405_16076_amd import OnlineRID, StreamConfig
    rng = np.random.default_rng(29)
    n, ell = 5 * t, 2 * t
    if growth == "dyn":
        A = (rng.standard_normal((n, m)) * 2.0 ** rng.uniform(-40, 40, (n, m))).astype(dtype)
    else:
        A = (rng.standard_normal((n, m)) * (growth ** np.arange(n))[:, None]).astype(dtype)
    dt = torch.float64 if dtype == np.float64 else torch.float32
    sk = "f64" if dtype == np.float64 else "f32"
    cfg = StreamConfig(m=m, ell=ell, k=t, t=t, n_max=n, dtype=dt, sketch=sk, omega_seed=51, select_seed=52,
                       gram=gram)
    s = OnlineRID(cfg)
    ld = (m + 15) // 16 * 16  # borrowed columns start on 64-byte boundaries
    Xp = torch.zeros((n, ld), dtype=dt, device="cuda:0")
    Xp[:, :m] = torch.from_numpy(A).to("cuda:0")
    X = Xp[:, :m]
    fills = []
    for u, j0 in enumerate(range(0, n, t)):
        s.push(X[j0:j0 + t], borrow=True)
        J = s.select()
        fills.append(s.update(u)["n_filled"])
        _, _, G = s.debug_state()
        _gram_check(G, A, J, "split" if gram == "split" else "exact", m, label=f"update {u}: ")
    log(f"  filled per update {fills}")
    assert any(0 < f < t for f in fills[1:]), fills


def test_gram_runs_equal_one_launch_per_update():
    # With the whole stream in one flush the split Grams of runs of updates
    # share a pass (the list of a run: the columns new at each update, latest
    # first, then the others occupied at its first); every entry keeps the
    # operands of its own update's launch, so G after every update, and with
    # it each NA-Hutch++ term, is bitwise that of one flush per update
    # (lookahead t).  The profile must show fewer Gram passes than updates
    # bringing columns, i.e. that runs formed.
    from paper_2405_16076_amd import OnlineRID, StreamConfig
    rng = np.random.default_rng(37)
    m, n, ell, t = 12_007, 640, 128, 64
    A = (rng.standard_normal((n, m)) * (1.02 ** np.arange(n))[:, None]).astype(np.float32)
    ld = (m + 15) // 16 * 16
    Xp = torch.zeros((n, ld), dtype=torch.float32, device="cuda:0")
    Xp[:, :m] = torch.from_numpy(A).to("cuda:0")
    X = Xp[:, :m]
    out = {}
    for la in (t, n):
        cfg = StreamConfig(m=m, ell=ell, k=t, t=t, n_max=n, dtype=torch.float32, sketch="f32", omega_seed=61,
                           select_seed=62, lookahead=la, gram="split")
        s = OnlineRID(cfg)
        s.profile_enable(True)
        for j0 in range(0, n, t):
            s.push(X[j0:j0 + t], borrow=True)
        s.finalize()
        prof = s.profile_read()
        nu = int(s.info().n_updates)
        recs = [s.update(u) for u in range(nu)]
        _, _, G = s.debug_state()
        out[la] = (s.select(), s.coefficients(), recs, G, prof)
        s.close()
    J0, P0, R0, G0, p0 = out[t]
    J1, P1, R1, G1, p1 = out[n]
    fills = [r["n_filled"] for r in R0]
    log(f"  filled per update {fills}; Gram passes {int(p0['gram_launches'])} one flush per update, "
        f"{int(p1['gram_launches'])} in one flush")
    assert np.array_equal(J0, J1) and np.array_equal(P0, P1) and np.array_equal(G0, G1)
    for a, b in zip(R0, R1):
        for key in ("F", "sk2", "lam", "E2", "tr_est", "gpp", "term1", "h", "corr"):
            assert a[key] == b[key], (a["update"], key, a[key], b[key])
    assert sum(f > 0 for f in fills) == int(p0["gram_launches"])
    assert int(p1["gram_launches"]) < int(p0["gram_launches"]), (fills, p0["gram_launches"], p1["gram_launches"])
    _gram_check(G1, A, J1, "split", m)


@pytest.mark.parametrize("growth,gram", [(1.0, "split"), (1.03, "split"), (1.03, "exact")])
def test_gram_incremental_matches_exact_products(growth, gram):
    # G is built incrementally over several updates (all-new first update, then
    # new x occupied blocks, possibly two tile groups when many slots refill);
    # after the last update it must equal A_J^T A_J of the final J.  Columns
    # growing in norm make old columns lose leverage, so many slots refill.
    rng = np.random.default_rng(23)
    m, n, ell, t = 20_011, 600, 300, 150
    A = (rng.standard_normal((n, m)) * (growth ** np.arange(n))[:, None]).astype(np.float32)
    s = run_gpu(A, ell, t, t, "f32", 41, 42, batch=100, gram=gram)
    info = s.info()
    fills = [s.update(u)["n_filled"] for u in range(int(info.n_updates))]
    log(f"  growth {growth}: filled per update {fills}")
    _, _, G = s.debug_state()
    _gram_check(G, A, s.select(), gram, m)
