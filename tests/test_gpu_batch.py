"""GPU tests of batched streams (rid_init_batch / rid_push_batch /
rid_finalize_batch), through the C ABI.

Every member of a batch is an ordinary stream with its own configuration and
seeds, so each member is checked against the oracle run on that member's
columns alone, with the same tolerances as the single-stream pipelines
(J exactly; S, P and a reconstruction within the fixed bounds of each form;
tau and the NA-Hutch++ terms within the oracle's forward-error tolerances).  Launch variants of the same batch (graph
capture or direct launches, COPY or BORROW pushes) must agree bitwise.
"""
import math

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


# members of uneven size and shape: (h, w, ell, t, n, push size per round)
MEMBERS = [(27, 37, 40, 20, 150, 25), (64, 64, 40, 20, 170, 7), (111, 111, 64, 32, 160, 40),
           (150, 200, 200, 50, 210, 33), (200, 328, 40, 20, 130, 64)]


def _frames(h, w, n, seed):
    """(n, ld) device tensor of blob frames (rows 16-byte aligned) and the
    host copy of its [:, :m] part."""
    A = synth.blobs(h, w, n, seed)
    m = h * w
    ld = (m + 15) // 16 * 16
    X = torch.zeros((n, ld), dtype=torch.float32, device="cuda:0")
    X[:, :m] = torch.from_numpy(A).to("cuda:0")
    return X, A


def _configs(sketch, lookahead, tile="auto"):
    from paper_2405_16076_amd import StreamConfig
    dt = torch.float64 if sketch == "f64" else torch.float32
    cfgs = []
    for i, (h, w, ell, t, n, _) in enumerate(MEMBERS):
        wide_ok = sketch == "bf16" and 128 < ell <= 320
        cfgs.append(StreamConfig(m=h * w, ell=ell, k=t, t=t, n_max=n, dtype=dt, sketch=sketch,
                                 omega_seed=4000 + i, select_seed=5000 + i, lookahead=lookahead,
                                 tile=tile if wide_ok else "auto"))
    return cfgs


def _run_batch(sketch, data, graph=True, tune=True, borrow=True, lookahead=0, tile="auto"):
    from paper_2405_16076_amd import StreamBatch
    if sketch == "f64":
        data = [(X.double(), A.astype(np.float64)) for X, A in data]
    B = StreamBatch(_configs(sketch, lookahead, tile), graph=graph, tune=tune)
    pos = [0] * len(MEMBERS)
    while any(p < mb[4] for p, mb in zip(pos, MEMBERS)):
        cols = []
        for i, (h, w, ell, t, n, step) in enumerate(MEMBERS):
            c = min(step, n - pos[i])
            cols.append(data[i][0][pos[i]:pos[i] + c, :h * w] if c > 0 else None)
            pos[i] += c
        B.push(cols, borrow=borrow)
    B.finalize()
    torch.cuda.synchronize()
    return B


@pytest.fixture(scope="module")
def data():
    return [_frames(h, w, n, synth.data_seed(4) + 17 * i) for i, (h, w, _, _, n, _) in enumerate(MEMBERS)]


def _check_member(mbr, A, ell, t, sketch, oseed, sseed, workers=1):
    o = run_oracle(A, ell, t, t, sketch, oseed, sseed, workers=workers)
    tol = perturbation_tolerances(o, A, sketch)
    worst_tau, margin = compare_updates(mbr, o, tol)
    J = mbr.select()
    assert np.array_equal(J, o.J)
    P = mbr.coefficients()
    occ = J >= 0
    assert np.allclose(P[occ][:, J[occ]], np.eye(int(occ.sum())), atol=1e-9 if sketch == "f64" else 1e-5)
    for u, rec in enumerate(o.records):
        g = mbr.update(u)
        for key in ("tr_est", "gpp", "E2"):
            assert abs(g[key] - rec.hutch[key]) <= tol[key][u], (u, key)
    n = A.shape[0]
    c0, c = max(0, n // 2 - 5), min(11, n)
    R = mbr.reconstruct(c0, c).cpu().numpy().astype(np.float64)
    Ro = (A.T[:, J[occ]].astype(np.float64) @ o.P[occ][:, c0:c0 + c]).T
    S, _, _ = mbr.debug_state()
    e, er = check_fixed_bounds(sketch, S[:, :o.n_obs], o.S[:, :o.n_obs], P, o.P, R, Ro, o.records[-1].cond_SJ, tol)
    return worst_tau, margin, e, er


@pytest.mark.parametrize("sketch,tile", [("f32", "auto"), ("bf16", "auto"), ("bf16", "wide"), ("fp8", "auto"),
                                        ("f64", "auto")])
def test_batch_members_match_oracle(sketch, tile, data):
    log(f"batch of {len(MEMBERS)} uneven members, {sketch} sketch ({tile} split where it applies), lookahead 64")
    B = _run_batch(sketch, data, lookahead=64, tile=tile)
    info = B.info()
    log(f"  info {info}")
    assert info["tuned"] == 1 and info["slab_rows"] in (2048, 4096, 8192, 16384, 32768, 65536)
    assert info["graph_launches"] == info["rounds"] and info["graph_updates"] >= 1
    assert info["wide"] == (1 if tile == "wide" else 0)
    for i, (h, w, ell, t, n, _) in enumerate(MEMBERS):
        A = data[i][1].astype(np.float64) if sketch == "f64" else data[i][1]
        wt, mg, e, er = _check_member(B.members[i], A, ell, t, sketch, 4000 + i, 5000 + i)
        log(f"  member {i} m={h * w} l={ell} t={t}: tau/tol {wt:.2e} margin {mg:.2e} P {e:.2e} recon {er:.2e}")
    B.close()


def _state(B):
    out = []
    for mbr in B.members:
        S, q, G = mbr.debug_state()
        out.append((S, q, G, mbr.select(), mbr.coefficients(), mbr.error_estimate()["E2"]))
    return out


def _same(a, b):
    for x, y in zip(a, b):
        for u, v in zip(x[:5], y[:5]):
            assert np.array_equal(u, v)
        assert x[5] == y[5]


def test_batch_graph_equals_direct_launches(data):
    log("graph-captured rounds against direct launches (bf16, default slab)")
    Bg = _run_batch("bf16", data, graph=True, tune=False, lookahead=40)
    ig = Bg.info()
    Bd = _run_batch("bf16", data, graph=False, tune=False, lookahead=40)
    idr = Bd.info()
    log(f"  graph {ig}\n  direct {idr}")
    assert ig["graph_launches"] == ig["rounds"] >= 5 and ig["graph_updates"] >= 1
    assert idr["graph_launches"] == 0 and idr["rounds"] == ig["rounds"]
    _same(_state(Bg), _state(Bd))
    Bg.close()
    Bd.close()


def test_batch_copy_equals_borrow(data):
    log("COPY pushes against BORROW pushes (f32)")
    Bb = _run_batch("f32", data, borrow=True, tune=False, lookahead=40)
    Bc = _run_batch("f32", data, borrow=False, tune=False, lookahead=40)
    _same(_state(Bb), _state(Bc))
    Bb.close()
    Bc.close()


def test_batch_member_rejects_direct_use(data):
    from paper_2405_16076_amd import _lib
    B = _run_batch("f32", data, tune=False)
    mbr = B.members[0]
    x = data[0][0][:1, :MEMBERS[0][0] * MEMBERS[0][1]]
    import ctypes as C
    lib = _lib.lib()
    assert lib.rid_push_snapshots(mbr._h, C.c_void_p(x.data_ptr()), x.stride(0), 1, _lib.RID_BORROW) == _lib.RID_ESTATE
    assert lib.rid_finalize(mbr._h) == _lib.RID_ESTATE
    assert lib.rid_destroy(mbr._h) == _lib.RID_ESTATE
    # the member still answers
    assert mbr.select().shape == (MEMBERS[0][3],)
    B.close()


def test_batch_image_streams_64_members_sampled():
    """64 image streams with m log-uniform in [1e4, 1e6] (l = 200, k = t = 100,
    bf16 sketch), 300 frames each pushed 100 per round.  Every member: J valid
    and distinct, P(:, J) = I, a finite estimate, logged beside the exact
    relative error of its reconstruction; the 16 members with m <= 20 000, the
    median member and the largest one against the oracle (J, tau, P, every
    NA-Hutch++ term including E^2, a reconstruction)."""
    from paper_2405_16076_amd import StreamBatch, StreamConfig
    shapes = synth.batch_frame_shapes(64, synth.data_seed(4))
    n, ell, t = 300, 200, 100
    log(f"64 members, sum m = {sum(h * w for h, w in shapes)}")
    X = [synth.blobs_torch(h, w, n, synth.data_seed(4) + 31 * i) for i, (h, w) in enumerate(shapes)]
    cfgs = [StreamConfig(m=h * w, ell=ell, k=t, t=t, n_max=n, dtype=torch.float32, sketch="bf16",
                         omega_seed=6000 + i, select_seed=7000 + i) for i, (h, w) in enumerate(shapes)]
    B = StreamBatch(cfgs)
    for j0 in range(0, n, 100):
        B.push([x[j0:j0 + 100, :h * w] for x, (h, w) in zip(X, shapes)], borrow=True)
    B.finalize()
    info = B.info()
    log(f"  info {info}")
    rows = []
    for i, mbr in enumerate(B.members):
        h, w = shapes[i]
        J = mbr.select()
        occ = J >= 0
        assert np.all(J[occ] < n) and len(set(J[occ].tolist())) == int(occ.sum())
        P = mbr.coefficients()
        assert P.shape == (t, n)
        assert np.allclose(P[occ][:, J[occ]], np.eye(int(occ.sum())), atol=1e-5)
        est = mbr.error_estimate()
        assert np.isfinite(est["E2"]) and est["n_obs"] == n
        A = X[i][:, :h * w]
        # the reconstruction is enqueued on the member's stream; the caller's
        # (null) stream must wait for it before the next operation reads R
        R = mbr.reconstruct(0, n)
        Pt = torch.from_numpy(P[occ]).to(A.device)                    # (|J|, n)
        Rref = Pt.T @ A[torch.from_numpy(J[occ]).to(A.device)].double()  # (n, m)
        assert float(torch.linalg.norm(R.double() - Rref) / torch.linalg.norm(Rref)) <= 1e-6
        exact = float(torch.linalg.norm((R.double() - A.double())) / torch.linalg.norm(A.double()))
        assert math.isfinite(exact)
        rows.append((h * w, est["E2"] / est["F"], est["rel"], exact))
        del R, Rref
    rows.sort()
    log("  m, E2 / F, estimate rel, exact rel:")
    for r in rows:
        log(f"    {r[0]:7d} {r[1]: .3e} {r[2]:.3e} {r[3]:.3e}")
    order = sorted(range(64), key=lambda i: shapes[i][0] * shapes[i][1])
    picked = [i for i in order if shapes[i][0] * shapes[i][1] <= 20_000] + [order[32], order[-1]]
    for i in picked:
        h, w = shapes[i]
        A = X[i][:, :h * w].cpu().numpy()
        wt, mg, e, er = _check_member(B.members[i], A, ell, t, "bf16", 6000 + i, 7000 + i, workers=8)
        log(f"  member {i} m={h * w}: tau/tol {wt:.2e} margin {mg:.2e} P {e:.2e} recon {er:.2e}")
    B.close()


def test_batch_many_updates_per_round_half_size_tridiagonalisation():
    """32 members with ten updates each in one round: 320 tridiagonalisation
    workgroups, more than one per compute unit, so they run at half the waves,
    two to a unit.  Every member: J valid and distinct, P(:, J) = I; every
    fourth member against the oracle."""
    from paper_2405_16076_amd import StreamBatch, StreamConfig
    n, ell, t = 240, 96, 24
    rng = np.random.default_rng(77)
    ms = [int(x) for x in rng.integers(2000, 9000, size=32)]
    data = []
    for i, m in enumerate(ms):
        A = synth.lowrank(m, n, seed=900 + i, rank=40)
        ld = (m + 15) // 16 * 16
        X = torch.zeros((n, ld), dtype=torch.float32, device="cuda:0")
        X[:, :m] = torch.from_numpy(A).to("cuda:0")
        data.append((X, A))
    cfgs = [StreamConfig(m=m, ell=ell, k=t, t=t, n_max=n, dtype=torch.float32, sketch="f32", omega_seed=8000 + i,
                         select_seed=8100 + i, lookahead=n) for i, m in enumerate(ms)]
    B = StreamBatch(cfgs)
    B.push([X[:, :m] for (X, _), m in zip(data, ms)], borrow=True)
    B.finalize()
    for i, mbr in enumerate(B.members):
        J = mbr.select()
        occ = J >= 0
        assert np.all(J[occ] < n) and len(set(J[occ].tolist())) == int(occ.sum())
        assert mbr.info().n_updates == n // t
        P = mbr.coefficients()
        assert np.allclose(P[occ][:, J[occ]], np.eye(int(occ.sum())), atol=1e-5)
    for i in range(0, 32, 4):
        wt, mg, e, er = _check_member(B.members[i], data[i][1], ell, t, "f32", 8000 + i, 8100 + i)
        log(f"  member {i} m={ms[i]}: tau/tol {wt:.2e} margin {mg:.2e} P {e:.2e} recon {er:.2e}")
    B.close()


def test_batch_coefficients_per_step_when_slices_do_not_fit():
    """A member whose per-update P slices (t x n_max each) would pass the cap
    gets each step's Alg. 4 / Alg. 8 phase right after that step's Gram (for
    every member of the round) instead of all at the end; every member still
    matches the oracle."""
    from paper_2405_16076_amd import StreamBatch, StreamConfig
    log("batch with an l = 400, t = 200, n_max = 400000 member: per-step coefficient phases")
    # binary64 form: the batch's default slab (16384 rows) sums a whole
    # 8192-row column in one partial, which binary32 would take past the
    # tolerances' model of the sketch error
    A1 = synth.lowrank(8192, 500, seed=synth.data_seed(5), rank=450, decay=300.0).astype(np.float64)
    A2 = synth.lowrank(5000, 300, seed=synth.data_seed(6), rank=30).astype(np.float64)
    cfgs = [StreamConfig(m=8192, ell=400, k=200, t=200, n_max=400_000, dtype=torch.float64, sketch="f64",
                         omega_seed=1005, select_seed=2005, lookahead=1024),
            StreamConfig(m=5000, ell=40, k=20, t=20, n_max=300, dtype=torch.float64, sketch="f64",
                         omega_seed=4001, select_seed=5001, lookahead=64)]
    B = StreamBatch(cfgs, tune=False)
    X1 = torch.from_numpy(A1).to("cuda:0")
    X2 = torch.from_numpy(A2).to("cuda:0")
    p1 = p2 = 0
    while p1 < 500 or p2 < 300:
        c1 = X1[p1:p1 + 100] if p1 < 500 else None
        c2 = X2[p2:p2 + 60] if p2 < 300 else None
        B.push([c1, c2])
        p1 += 100
        p2 += 60
    B.finalize()
    torch.cuda.synchronize()
    for i, (A, ell, t, os_, ss) in enumerate([(A1, 400, 200, 1005, 2005), (A2, 40, 20, 4001, 5001)]):
        wt, mg, e, er = _check_member(B.members[i], A, ell, t, "f64", os_, ss)
        log(f"  member {i}: tau/tol {wt:.2e} margin {mg:.2e} P {e:.2e} recon {er:.2e}")
    B.close()
