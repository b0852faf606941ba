"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on
the same seeded bytes and compare."""
from __future__ import annotations

import math
import sys

import numpy as np
import torch

import oracle
from oracle.rid import Config, OnlineRID as OracleRID


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(A_cols, ell, k, t, sketch, omega_seed, select_seed, batch=None, borrow=True, lookahead=0,
            finalize=True, n1=0, n2=0, tile="auto", n_max=None, coeff="alg4", gram="auto"):
    """A_cols: numpy (n, m) (row j = snapshot j).  Returns the stream after
    pushing every snapshot (and finalizing)."""
    from paper_2405_16076_amd import OnlineRID, StreamConfig
    n, m = A_cols.shape
    dt = torch.float64 if A_cols.dtype == np.float64 else torch.float32
    cfg = StreamConfig(m=m, ell=ell, k=k, t=t, n_max=n_max or n, dtype=dt, sketch=sketch, omega_seed=omega_seed,
                       select_seed=select_seed, lookahead=lookahead, hutch_n1=n1, hutch_n2=n2, tile=tile,
                       coeff=coeff, gram=gram)
    s = OnlineRID(cfg)
    # padded device copy: every column starts on a 64-byte boundary
    ld = (m + 15) // 16 * 16
    Xp = torch.zeros((n, ld), dtype=dt, device="cuda:0")
    Xp[:, :m] = torch.from_numpy(A_cols).to("cuda:0")
    X = Xp[:, :m]
    batch = batch or n
    for j0 in range(0, n, batch):
        s.push(X[j0:j0 + batch], borrow=borrow)
    if finalize:
        s.finalize()
    torch.cuda.synchronize()
    s._data = X
    return s


def run_oracle(A_cols, ell, k, t, sketch, omega_seed, select_seed, finalize=True, n1=None, n2=None, workers=1,
               coeff="alg4"):
    n, m = A_cols.shape
    operand = {"f64": "f64", "f32": "f32", "bf16": "bf16", "fp8": "fp8"}[sketch]
    cfg = Config(m=m, ell=ell, k=k, t=t, omega_seed=omega_seed, select_seed=select_seed, operand=operand,
                 hutch_n1=n1, hutch_n2=n2, workers=workers, coeff=coeff)
    o = OracleRID(cfg, n_max=n)
    o.push(A_cols.T)
    if finalize:
        o.finalize()
    return o


def rel_fro(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def col_max_rel(a, b):
    """Largest |a - b| in each column divided by that column's norm of b
    (the worst column)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.max(np.abs(a - b), axis=0) if a.size else np.zeros(0)
    nb = np.linalg.norm(b, axis=0)
    return float(np.max(d / np.where(nb > 0, nb, 1.0))) if d.size else 0.0


def compare_updates(s, o, tol, log_prefix=""):
    """J of every update must match exactly; tau within the per-update
    tolerance.  Returns the worst tau ratio (diff / tolerance) and the smallest
    decision margin."""
    worst = 0.0
    min_margin = math.inf
    for u, rec in enumerate(o.records):
        g = s.update(u)
        mm = rec.min_margin()
        min_margin = min(min_margin, mm)
        if rec.tau_D is not None:
            d = float(np.max(np.abs(g["tau_D"] - rec.tau_D) / np.maximum(np.abs(rec.tau_D), 1e-300)))
            occ = ~np.isnan(rec.tau_C)
            if occ.any():
                d = max(d, float(np.max(np.abs(g["tau_C"][occ] - rec.tau_C[occ]) / np.abs(rec.tau_C[occ]))))
            worst = max(worst, d / tol["tau"][u])
            assert d <= tol["tau"][u], (u, d, tol["tau"][u])
        if not np.array_equal(g["J"], rec.J):
            raise AssertionError(f"{log_prefix} J differs at update {u}: min margin {mm:.3e}\n"
                                 f" gpu {g['J']}\n orc {rec.J}")
        assert g["n_filled"] == rec.n_filled and g["n_pruned"] == rec.n_pruned, (u, g, rec.n_filled, rec.n_pruned)
    return worst, min_margin


# Relative accuracy of the sketch S of each form against the oracle's S of the
# same operands (the test matrices are equal bit for bit): binary64 sums in
# another order (~sqrt(m) 2^-53); binary32 accumulation within a slab (~1e-6;
# the bfloat16 form's slabs of up to 64k rows are modelled at 5e-6); e4m3
# operands: the scaled MFMA rounds inside each 64-term product (a few 1e-5 of
# the sum of magnitudes, ~1e-4 of S).
SKETCH_ACCURACY = {"f64": 1e-14, "f32": 1e-6, "bf16": 5e-6, "fp8": 3e-4}

# Fixed bounds on the coefficients P and the reconstruction A_J P, declared
# before any GPU value is seen: relative Frobenius norm of the difference from
# the oracle's, and the worst column (largest |difference| in a column over
# that column's norm).  The oracle multiplies the same rounded operands as the
# form (bfloat16, e4m3 with the same block scales), so these bound the
# arithmetic of the HIP path, not the rounding of the data.
#
# P's forward error is about cond(Omega A_J) times the relative error of the
# sketch S (binary64 ~1e-15, binary32 ~3e-7, bfloat16 ~2e-5, e4m3 ~4e-4 of the
# oracle's product of the same operands).  Binary32 P is held to 1e-5 when
# Omega A_J has condition number <= 100; above that (the channel and image
# streams: 1e3 and more) P is held to 1e-3 and the better-conditioned
# reconstruction A_J P to 1e-5.
P_BOUND = {"f64": 1e-10, "f32": 1e-5, "bf16": 1e-3, "fp8": 3e-3}
P_BOUND_F32_ILL_CONDITIONED = 1e-3
F32_WELL_CONDITIONED = 100.0
# the worst column of P: binary64 columns of small norm carry relative errors
# above the matrix's (cond(Omega A_J) up to 2e4 times 1e-15 of S)
P_COL_FACTOR = {"f64": 10.0, "f32": 1.0, "bf16": 1.0, "fp8": 1.0}
RECON_BOUND = {"f64": 1e-10, "f32": 1e-5, "bf16": 1e-4, "fp8": 1e-3}
# worst column of S against the oracle's S of the same operands (the test
# matrices are equal bit for bit; what is left is the accumulation: binary64,
# or binary32 within a row slab, and the e4m3 matrix cores' internal rounding)
S_COL_BOUND = {"f64": 1e-13, "f32": 2e-6, "bf16": 2e-6, "fp8": 2e-3}


def p_bound(sketch, cond_SJ):
    if sketch == "f32" and not cond_SJ <= F32_WELL_CONDITIONED:
        return P_BOUND_F32_ILL_CONDITIONED
    return P_BOUND[sketch]


def check_fixed_bounds(sketch, S, So, P, Po, R, Ro, cond_SJ, tol=None, prefix="  ", pb=None, rb=None):
    """Asserts the fixed bounds above on S (worst column), P (relative
    Frobenius and worst column) and the reconstruction; logs the measured
    values, the bound and (if given) the oracle-derived forward-error
    tolerance as a diagnostic.  pb / rb replace the form's P and
    reconstruction bounds where a test declares its own."""
    es, ecs = rel_fro(S, So), col_max_rel(S, So)
    ep, ecp = rel_fro(P, Po), col_max_rel(P, Po)
    er, ecr = rel_fro(R, Ro), col_max_rel(R.T, Ro.T)
    pb = pb or p_bound(sketch, cond_SJ)
    rb = rb or RECON_BOUND[sketch]
    diag = f" (derived {tol['P']:.2e} / {tol['recon']:.2e})" if tol else ""
    log(f"{prefix}S rel fro {es:.2e} col {ecs:.2e} (bound {S_COL_BOUND[sketch]:.0e}); "
        f"P rel fro {ep:.2e} col {ecp:.2e} (bound {pb:.0e}, cond S_J {cond_SJ:.2e}); "
        f"recon rel fro {er:.2e} col {ecr:.2e} (bound {rb:.0e}){diag}")
    assert ecs <= S_COL_BOUND[sketch], ("S column", ecs)
    assert ep <= pb and ecp <= P_COL_FACTOR[sketch] * pb, ("P", ep, ecp, pb)
    assert er <= rb and ecr <= rb, ("reconstruction", er, ecr, rb)
    return ep, er


# Relative accuracy of the basis Gram G = A_J^T A_J: products of the data are
# exact in binary64 and the sums are binary64 (another order than the oracle).
GRAM_ACCURACY = {"f64": 1e-15, "f32": 1e-15, "bf16": 1e-15, "fp8": 1e-15}


def gram_split_eps(m):
    """The library's elementwise bound of the split-form Gram, relative to
    sum_r |a_ri| |a_rj| (three-piece bfloat16 split, order <= 2 products,
    binary32 sums over 32 rows counted as rounded at every addition, then
    binary64 over at most m / 64 + 1024 additions; m / 32 kept as the margin)."""
    return 37 * 2.0 ** -24 + (m / 32 + 1024) * 2.0 ** -53


def uses_gram_split(sketch, coeff="alg4", gram="auto"):
    """Whether a stream of this form and modes forms G in the split form."""
    return sketch != "f64" and (gram == "split" or (gram == "auto" and coeff == "alg4"))


def split_gram_bounds(S, SJ, P, G, n1, n2, m, occ):
    """Bounds on how far the split form's G moves the two NA-Hutch++ terms
    that use it (Alg. 8): term1 = tr(K^+ Y1 G Y2^T) = sum_ij G_ij B_ji with
    B = Y2^T K^+ Y1, and gpp = sum_ij G_ij (P P^T)_ij.  With
    |dG_ij| <= eps sqrt(G_ii G_jj) (Cauchy-Schwarz on sum_r |a_ri||a_rj|),
    |d term| <= eps sum_ij sqrt(G_ii G_jj) |C_ij|.  Returns (term1, gpp)."""
    if not occ.size:
        return 0.0, 0.0
    eps = gram_split_eps(m)
    dg = np.sqrt(np.abs(np.diag(G)))[occ]
    Pk = P[occ]
    b_gpp = eps * float(dg @ np.abs(Pk @ Pk.T) @ dg)
    b_t1 = 0.0
    if n1 and n2:
        W = SJ @ P
        K = S[:n1] @ W[n1:n1 + n2].T
        B = (S[n1:n1 + n2] @ Pk.T).T @ np.linalg.pinv(K) @ (S[:n1] @ Pk.T)
        b_t1 = eps * float(dg @ np.abs(B.T) @ dg)
    return b_t1, b_gpp


def hutch_regrouped(S, SJ, P, G, F, n1, n2):
    """The NA-Hutch++ terms of the oracle's formula with the same products
    grouped another way (through Y = S P^T and P P^T).  Mathematically equal;
    the spread between the two groupings measures how much rounding inside the
    formula itself can move the result."""
    from oracle.rid import pinv
    ell = S.shape[0]
    n3 = ell - n1 - n2
    Y = S @ P.T
    Y1, Y2, Y3 = Y[:n1], Y[n1:n1 + n2], Y[n1 + n2:]
    SJ2, SJ3 = SJ[n1:n1 + n2], SJ[n1 + n2:]
    Kp = pinv(Y1 @ SJ2.T)
    term1 = float(np.trace(Kp @ (Y1 @ G @ Y2.T)))
    corr = float(np.trace(Kp @ ((Y1 @ SJ3.T) @ (SJ3 @ Y2.T))))
    h = float(np.sum(Y3 * SJ3))
    tr_est = term1 + (h - corr) / n3
    gpp = float(np.sum(G * (P @ P.T)))
    return dict(tr_est=tr_est, gpp=gpp, E2=F - 2.0 * tr_est + gpp)


def exact_gram(A_cols, idx, chunk=1 << 20):
    """A_J^T A_J in binary64 for the snapshots (rows of A_cols) listed in idx,
    summed over chunks of the snapshot rows (binary32 products are exact)."""
    idx = np.asarray(idx)
    G = np.zeros((idx.size, idx.size))
    if idx.size == 0:
        return G
    m = A_cols.shape[1]
    for i0 in range(0, m, chunk):
        X = A_cols[idx, i0:i0 + chunk].astype(np.float64)
        G += X @ X.T
    return G


def perturbation_tolerances(o, A_cols, sketch, draws=3, factor=10.0, seed=0, recon=True, gram="auto"):
    """Forward-error tolerances derived from the conditioning of each step.

    The oracle's own S is perturbed column by column at the sketch accuracy of
    the form; tau, P, the NA-Hutch++ terms and the reconstruction are
    recomputed with the oracle's functions; for the NA-Hutch++ terms the spread
    between two groupings of the same products is included as well.  The
    tolerance is `factor` times the largest change seen (plus a floor at the
    binary64 rounding level).  Where the stream forms G in the split form, the
    tr_est, gpp and E2 tolerances also take that form's bounds on the two
    terms that use G (split_gram_bounds).  No GPU value enters."""
    from oracle.rid import coeff_alg4, nahutchpp, ridge_lambda, ridge_scores
    rng = np.random.default_rng(seed)
    cfg = o.cfg
    u_S = SKETCH_ACCURACY[sketch]
    tol = {"tau": [], "tr_est": [], "gpp": [], "E2": [], "b_term1": []}
    split = uses_gram_split(sketch, getattr(cfg, "coeff", "alg4"), gram)
    S_full = o.S[:, :o.n_obs]
    norms = np.linalg.norm(S_full, axis=0) / np.sqrt(cfg.ell)
    perturbed = [S_full + u_S * norms * rng.standard_normal(S_full.shape) for _ in range(draws)]
    for rec in o.records:
        n = rec.n_obs
        S = S_full[:, :n]
        J = rec.J
        occ = np.flatnonzero(J >= 0)
        G = np.zeros((cfg.t, cfg.t))
        if occ.size:
            G[np.ix_(occ, occ)] = exact_gram(A_cols, J[occ])
        u_G = GRAM_ACCURACY[sketch]
        dg = np.sqrt(np.abs(np.diag(G)))
        P0 = coeff_alg4(S, J)
        SJ0 = np.zeros((cfg.ell, cfg.t)); SJ0[:, occ] = S[:, J[occ]]
        h0 = nahutchpp(S, SJ0, P0, G, rec.F, cfg.n1, cfg.n2)
        hr = hutch_regrouped(S, SJ0, P0, G, rec.F, cfg.n1, cfg.n2)
        dtr = abs(hr["tr_est"] - h0["tr_est"])
        dgpp = abs(hr["gpp"] - h0["gpp"])
        dE2 = abs(hr["E2"] - h0["E2"])
        dtau = 0.0
        for Sp_full in perturbed:
            Sp = Sp_full[:, :n]
            if rec.tau_D is not None:
                SST = Sp @ Sp.T
                _, lam, _ = ridge_lambda(SST, rec.F, cfg.k, cfg.ell, cfg.ridge_floor)
                cols = list(range(n - rec.count, n))
                tD = ridge_scores(SST, lam, cfg.ell, Sp[:, cols])
                dtau = max(dtau, float(np.max(np.abs(tD - rec.tau_D) / rec.tau_D)))
            Pp = coeff_alg4(Sp, J)
            SJp = np.zeros((cfg.ell, cfg.t)); SJp[:, occ] = Sp[:, J[occ]]
            xi = rng.standard_normal(G.shape)
            Gp = G + u_G * np.outer(dg, dg) * (xi + xi.T) / 2
            hp = nahutchpp(Sp, SJp, Pp, Gp, rec.F, cfg.n1, cfg.n2)
            dtr = max(dtr, abs(hp["tr_est"] - h0["tr_est"]))
            dgpp = max(dgpp, abs(hp["gpp"] - h0["gpp"]))
            dE2 = max(dE2, abs(hp["E2"] - h0["E2"]))
        floor = 1e-11 * max(rec.F, 1e-300)
        b_t1 = b_gpp = 0.0
        if split:
            b_t1, b_gpp = split_gram_bounds(S, SJ0, P0, G, cfg.n1, cfg.n2, A_cols.shape[1], occ)
        tol["b_term1"].append(b_t1)
        tol["tau"].append(factor * dtau + 1e-12)
        tol["tr_est"].append(factor * dtr + floor + b_t1)
        tol["gpp"].append(factor * dgpp + floor + b_gpp)
        tol["E2"].append(factor * dE2 + 2 * floor + 2 * b_t1 + b_gpp)
    # final coefficients and reconstruction
    Pn = o.P
    dP = dR = 0.0
    J = o.J
    occ = np.flatnonzero(J >= 0)
    AJ = A_cols[J[occ]].T.astype(np.float64) if recon else None
    R0 = AJ @ Pn[occ] if recon else None
    for Sp_full in perturbed:
        Pp = coeff_alg4(Sp_full, J)
        dP = max(dP, float(np.linalg.norm(Pp - Pn) / max(np.linalg.norm(Pn), 1e-300)))
        if recon:
            Rp = AJ @ Pp[occ]
            dR = max(dR, float(np.linalg.norm(Rp - R0) / max(np.linalg.norm(R0), 1e-300)))
    tol["P"] = factor * dP + 1e-12
    tol["recon"] = factor * dR + 1e-7 if sketch != "f64" else factor * dR + 1e-12
    return tol
