"""CPU oracle of the single-pass online randomized ID (test infrastructure only).

Plain, slow, binary64 code that follows the paper step by step.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg use it; the
product path (the HIP library and its binding) never imports it, and this
module imports nothing from the product path.

What it computes (Li, Becker, Doostan, "Single-pass randomized ID"):

* Alg. 3 (single-pass randomized ID): per snapshot a_j, the sketch
  s_j = Omega a_j, SS^T += s_j s_j^T, ||A_obs||_F^2 += ||a_j||^2 and buffering
  into D; when t columns are buffered, ridge leverage scores of the basis C and
  the buffer D (eq. ``sketch_ridge_leverage_score``), the reservoir-style
  prune/fill of the basis, then the coefficients and the error estimate.
* Alg. 4 (eq. ``coeff_rID_fullsketch``): P = (Omega A_J)^+ (Omega A_obs).
* Alg. 8 with eqs. ``NAhutchPP_expansion`` and ``NAhutchPP_2nd_term``:
  the NA-Hutch++ estimate of ||A_obs - A_J P||_F^2.

Readings taken where the paper is silent or garbled (each is listed, with its
reason, in the design notes of the repository):

* Omega has unit-variance entries (Alg. 3 step 2, Sec. 3.3), so the sketch
  carries l times the energy of the data; the scores are taken with the
  normalised sketch Omega / sqrt(l): tau = s^T (SS^T + l*lam I)^{-1} s.
* The ridge parameter: the printed ridge term (||A_obs||_F^2 - ||S_k||_F^2)/k
  estimates the rank-k tail energy over k (eq. ridge-leverage-score).  The
  sketch's top-k energy is put on the scale of F through the sketch's own
  total energy, lam = max(F (1 - ||S_k||^2 / ||S||^2) / k, rho F / k): the
  tail fraction of the sketch itself, as the generalised score of
  eq. g_ridge_leverage_score takes ||B - B_k||^2 from the sketch B.  It is
  never negative and needs no difference of two independently estimated
  energies (F against ||S_k||^2 / l), which sketch noise makes cancel.
* S holds every observed column (l x n_obs), not l x t.
* The update fires right after the t-th buffered column (and its norm) has
  been added; a partial buffer is flushed by ``finalize``.
* Fill step: slot by slot, scan the buffer in arrival order, skip columns
  already placed in this update, and the first successful draw fills the slot.
* A draw "with probability p" succeeds iff U < p, U a 53-bit uniform.
* Alg. 4 is solved over the occupied slots with an SVD pseudo-inverse; rows of
  empty slots are zero.
* NA-Hutch++ uses the contiguous row split [0,n1), [n1,n1+n2), [n1+n2,l) with
  n1 = l//4, n2 = l//2 by default, and the formula of eq. NAhutchPP_2nd_term
  as printed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .omega import omega_block, quantize_fp8_blocks, quantize_fp8_omega, round_to_bf16
from .philox import PRUNE_DRAW, decision_uniform


@dataclass
class Config:
    m: int
    ell: int
    k: int
    t: int
    omega_seed: int = 1
    select_seed: int = 2
    delta: float = 0.05        # success probability 1 - delta (Sec. 4.1 channel flow)
    eps: float = 0.5           # accuracy epsilon (Sec. 4.1 channel flow)
    c_sample: float = 1.0      # the constant c of the fill probability
    ridge_floor: float = 1e-8  # rho of the ridge floor
    hutch_n1: int | None = None
    hutch_n2: int | None = None
    operand: str = "f64"       # operand rounding of the sketch: f64, f32, bf16 or fp8
    row_chunk: int = 1 << 16   # rows of Omega regenerated at a time
    workers: int = 1           # threads that compute the sketch's row chunks
    coeff: str = "alg4"        # "alg4": Alg. 4 at every update; "best4": the best of Algs. 4-7

    @property
    def n1(self):
        return self.ell // 4 if self.hutch_n1 is None else self.hutch_n1

    @property
    def n2(self):
        return self.ell // 2 if self.hutch_n2 is None else self.hutch_n2

    @property
    def n3(self):
        return self.ell - self.n1 - self.n2


def fill_factor(cfg):
    """c (k ln k + k ln(1/delta)/eps) / t: the factor multiplying tau^D in the
    fill probability (Alg. 3 fill step; the bound on t in Sec. 2.2.2)."""
    k = cfg.k
    return cfg.c_sample * (k * math.log(k) + k * math.log(1.0 / cfg.delta) / cfg.eps) / cfg.t


# --------------------------------------------------------------------------
# Sketch (eq. random_sketch; Alg. 3 steps 10-13)
# --------------------------------------------------------------------------

def _round_operand(x, operand):
    if operand == "f64":
        return np.asarray(x, dtype=np.float64)
    if operand == "f32":
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    if operand == "bf16":
        return round_to_bf16(x)
    raise ValueError(f"unknown operand rounding {operand!r}")


def _sketch_chunk(cols, omega_seed, ell, operand, i0, n):
    """Omega(:, i0:i0+n) A(i0:i0+n, :) and the chunk's sum of squares per column."""
    blk = cols[i0:i0 + n].astype(np.float64)
    om = omega_block(omega_seed, ell, i0, n)
    if operand == "fp8":
        # e4m3 operands: Omega with the fixed scale 2^-6, the data with one
        # power-of-two scale per 32 rows of each column (row_chunk is a
        # multiple of 32, so the blocks stay aligned to row 0)
        part = quantize_fp8_omega(om) @ quantize_fp8_blocks(blk)
    else:
        part = _round_operand(om, operand) @ _round_operand(blk, operand)
    return part, np.einsum("ij,ij->j", blk, blk)


def sketch_columns(cols, omega_seed, ell, operand="f64", row_chunk=1 << 16, workers=1):
    """S = Omega A for the columns of ``cols`` (m x b), and ||a_j||^2.

    Omega is regenerated block by block from its counter.  ``operand`` names
    the rounding applied to both operands before the (exact binary64) product:
    the reduced-precision sketch forms multiply rounded operands.  Column norms
    are always those of the unrounded data, accumulated in binary64.

    The sum over row chunks is taken in chunk order.  With ``workers`` > 1 the
    chunks' products are computed by that many threads (numpy releases the
    interpreter lock inside its array loops) and still added in chunk order,
    so the result does not depend on ``workers``."""
    cols = np.asarray(cols)
    m, b = cols.shape
    if operand == "fp8" and row_chunk % 32:
        raise ValueError("row_chunk must be a multiple of 32 for the fp8 operands")
    S = np.zeros((ell, b), dtype=np.float64)
    colsq = np.zeros(b, dtype=np.float64)
    starts = list(range(0, m, row_chunk))

    def one(i0):
        return _sketch_chunk(cols, omega_seed, ell, operand, i0, min(row_chunk, m - i0))

    if workers <= 1 or len(starts) <= 1:
        for i0 in starts:
            part, sq = one(i0)
            S += part
            colsq += sq
        return S, colsq
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1), ThreadPoolExecutor(workers) as ex:
        # a bounded window of chunks in flight keeps the memory in check
        window = 2 * workers
        futs = [ex.submit(one, i0) for i0 in starts[:window]]
        nxt = window
        for k in range(len(starts)):
            part, sq = futs[k].result()
            futs[k] = None
            S += part
            colsq += sq
            if nxt < len(starts):
                futs.append(ex.submit(one, starts[nxt]))
                nxt += 1
    return S, colsq


# --------------------------------------------------------------------------
# Ridge leverage scores (eq. sketch_ridge_leverage_score; Alg. 3 function)
# --------------------------------------------------------------------------

def ridge_lambda(SST, F, k, ell, floor):
    """||S_k||_F^2 (sum of the top min(k, l) eigenvalues of SS^T) and the ridge
    parameter lam = max(F (tr(SS^T) - ||S_k||^2) / tr(SS^T) / k, floor*F/k)
    (the rank-k tail fraction of the sketch times F, over k; eqs.
    sketch_ridge_leverage_score and g_ridge_leverage_score).  ``ell`` only
    bounds the number of eigenvalues."""
    mu = np.linalg.eigvalsh(SST)[::-1]
    sk2 = float(np.sum(mu[:min(k, ell)]))
    tr = float(np.trace(SST))
    tail = F * (tr - sk2) / tr if tr > 0.0 else 0.0
    lam = max(tail / k, floor * F / k)
    return sk2, lam, mu


def ridge_scores(SST, lam, ell, cols_S):
    """tau_i = s_i^T (SS^T + l*lam*I)^{-1} s_i for the columns s_i of cols_S."""
    M = SST + (ell * lam) * np.eye(SST.shape[0])
    L = np.linalg.cholesky(M)
    Y = sla.solve_triangular(L, cols_S, lower=True)
    return np.sum(Y * Y, axis=0)


# --------------------------------------------------------------------------
# Prune / fill (Alg. 3 inner loop over slots)
# --------------------------------------------------------------------------

@dataclass
class Decision:
    kind: str      # "prune" or "fill"
    slot: int
    r: int
    p: float
    U: float
    success: bool


def select_slots(u, J, tau_old, tau_C, tau_D, d_idx, fill_mult, select_seed):
    """One pass of the prune/fill loop.

    J: slot -> snapshot index (-1 = empty); tau_C: current scores of the
    occupied slots (already min'ed with tau_old); tau_D, d_idx: scores and
    snapshot indices of the buffered columns in arrival order.
    Returns the new J, tau_old, the mask of slots filled in this update and the
    list of decisions taken."""
    J = np.array(J, dtype=np.int64).copy()
    tau_old = np.array(tau_old, dtype=np.float64).copy()
    t = J.shape[0]
    q = np.minimum(1.0, fill_mult * np.asarray(tau_D, dtype=np.float64))
    used = np.zeros(len(d_idx), dtype=bool)
    filled = np.zeros(t, dtype=bool)
    decisions = []
    for i in range(t):
        if J[i] >= 0:
            p = 1.0 - tau_C[i] / tau_old[i]
            U = float(decision_uniform(select_seed, u, i, PRUNE_DRAW))
            hit = U < p
            decisions.append(Decision("prune", i, -1, p, U, hit))
            if hit:
                J[i] = -1
                tau_old[i] = 1.0
            else:
                tau_old[i] = tau_C[i]
        if J[i] < 0:
            for r in range(len(d_idx)):
                if used[r]:
                    continue
                U = float(decision_uniform(select_seed, u, i, r))
                hit = U < q[r]
                decisions.append(Decision("fill", i, r, float(q[r]), U, hit))
                if hit:
                    J[i] = d_idx[r]
                    tau_old[i] = tau_D[r]
                    used[r] = True
                    filled[i] = True
                    break
    return J, tau_old, filled, decisions


# --------------------------------------------------------------------------
# Alg. 4 and Alg. 8
# --------------------------------------------------------------------------

def pinv(a):
    """Moore-Penrose pseudo-inverse by SVD; singular values at or below
    max(rows, cols) * eps * sigma_max are treated as zero."""
    a = np.asarray(a, dtype=np.float64)
    if a.size == 0:
        return np.zeros((a.shape[1], a.shape[0]))
    U, s, Vt = np.linalg.svd(a, full_matrices=False)
    cut = max(a.shape) * np.finfo(np.float64).eps * (s[0] if s.size else 0.0)
    inv = np.where(s > cut, 1.0 / np.where(s > cut, s, 1.0), 0.0)
    return (Vt.T * inv) @ U.T


def coeff_alg4(S, J):
    """P = (S_J)^+ S over the occupied slots of J (eq. coeff_rID_fullsketch);
    rows of empty slots are zero.  S is l x n_obs."""
    t = len(J)
    P = np.zeros((t, S.shape[1]))
    occ = np.flatnonzero(np.asarray(J) >= 0)
    if occ.size:
        SJ = S[:, np.asarray(J)[occ]]
        P[occ] = pinv(SJ) @ S
    return P


def nahutchpp(S, SJ, P, G, F, n1, n2):
    """NA-Hutch++ estimate of ||A_obs - A_J P||_F^2 (Alg. 8).

    S = Omega A_obs (l x n), SJ = Omega A_J (l x t), P (t x n), G = A_J^T A_J,
    F = ||A_obs||_F^2.  Rows [0,n1), [n1,n1+n2), [n1+n2,l) of Omega play the
    parts of Omega_1, Omega_2, Omega_3."""
    ell = S.shape[0]
    n3 = ell - n1 - n2
    W = SJ @ P
    S1, S2, S3 = S[:n1], S[n1:n1 + n2], S[n1 + n2:]
    W2, W3 = W[n1:n1 + n2], W[n1 + n2:]
    K = S1 @ W2.T
    Kp = pinv(K)
    Y1 = S1 @ P.T
    Y2 = S2 @ P.T
    term1 = float(np.trace(Kp @ Y1 @ G @ Y2.T)) if n1 and n2 else 0.0
    h = float(np.sum(S3 * W3))
    corr = float(np.trace(W3 @ S2.T @ Kp @ S1 @ W3.T)) if n1 and n2 else 0.0
    tr_est = term1 + (h - corr) / n3
    gpp = float(np.sum((G @ P) * P))
    e2 = F - 2.0 * tr_est + gpp
    return dict(E2=e2, tr_est=tr_est, gpp=gpp, term1=term1, h=h, corr=corr,
                E=math.sqrt(max(e2, 0.0)), rel=(math.sqrt(max(e2, 0.0)) / math.sqrt(F)) if F > 0 else 0.0)


# --------------------------------------------------------------------------
# Algs. 5-7 and the best of four (Alg. 3, coefficient steps)
# --------------------------------------------------------------------------

def _occupied(J):
    return np.flatnonzero(np.asarray(J) >= 0)


def coeff_alg5(S, J, G, ell):
    """Alg. 5 (partial sketching): P = G^{-1} Y over the occupied slots, with
    G = A_J^T A_J the exact basis Gram and Y = (Omega A_J)^T (Omega A_obs) / l
    (the sketch carries l times the data's inner products, reading R1); rows of
    empty slots are zero.  G^{-1} is the pseudo-inverse when G is singular."""
    t = len(J)
    P = np.zeros((t, S.shape[1]))
    occ = _occupied(J)
    if occ.size:
        SJ = S[:, np.asarray(J)[occ]]
        Y = SJ.T @ S / ell
        P[occ] = pinv(G[np.ix_(occ, occ)]) @ Y
    return P


def unchanged_slots(J, J_prev):
    """Slots holding the same snapshot before and after the update."""
    J, J_prev = np.asarray(J), np.asarray(J_prev)
    return (J >= 0) & (J == J_prev)


def coeff_alg6(S, J, J_prev, P_prev, literal=False):
    """Alg. 6 (residual of the fully sketched least squares) for the columns
    that P_prev covers (the first P_prev.shape[1] of S): rows of P_prev for
    slots that did not keep their column are zeroed (eq.
    coeff_update_residual_zeroout), r_A = S - S_J P_prev, and
    delta P = argmin ||S_J X - r_A|| is fitted over the new slots only (the
    text: the new basis elements fit the residual), or over every occupied
    slot (``literal``: the algorithm as printed, which equals Alg. 4 when S_J
    has full column rank); P = P_prev + delta P."""
    t = len(J)
    n_prev = P_prev.shape[1]
    S_old = S[:, :n_prev]
    keep = unchanged_slots(J, J_prev)
    Pz = np.where(keep[:, None], P_prev, 0.0)
    occ = _occupied(J)
    SJ = np.zeros((S.shape[0], t))
    SJ[:, occ] = S[:, np.asarray(J)[occ]]
    rA = S_old - SJ @ Pz
    fit = occ if literal else np.flatnonzero((np.asarray(J) >= 0) & ~keep)
    dP = np.zeros((t, n_prev))
    if fit.size:
        dP[fit] = pinv(SJ[:, fit]) @ rA
    return Pz + dP


def alg7_transform(C, J, C_prev, J_prev):
    """T = R^+ Q^T A_{J_prev} with A_J = Q R (Alg. 7): the coefficients of the
    previous basis columns in the current basis; rows for the current slots,
    columns for the previous slots (zero for empty slots).  C and C_prev hold
    the basis columns by slot (m x t)."""
    t = len(J)
    T = np.zeros((t, len(J_prev)))
    occ, occ_p = _occupied(J), _occupied(J_prev)
    if occ.size and occ_p.size:
        AJ = C[:, occ].astype(np.float64)
        Q, R = np.linalg.qr(AJ)
        T[np.ix_(occ, occ_p)] = pinv(R) @ (Q.T @ C_prev[:, occ_p].astype(np.float64))
    return T


def coeff_alg7(T, P_prev):
    """Alg. 7: P = T P_prev for the columns P_prev covers."""
    return T @ P_prev


# --------------------------------------------------------------------------
# The streaming driver (Alg. 3)
# --------------------------------------------------------------------------

@dataclass
class UpdateRecord:
    u: int
    n_obs: int
    count: int
    F: float
    sk2: float = float("nan")
    lam: float = float("nan")
    skipped: bool = False
    tau_C: np.ndarray | None = None
    tau_D: np.ndarray | None = None
    J: np.ndarray | None = None
    filled: np.ndarray | None = None
    n_pruned: int = 0
    n_filled: int = 0
    decisions: list = field(default_factory=list)
    hutch: dict | None = None
    e2_q: list | None = None        # best4: the NA-Hutch++ estimate of Algs. 4, 5, 6, 7
    q_star: int = 4                 # the algorithm whose coefficients were kept
    kappa: float = float("nan")     # cond(SS^T + l lam I): diagnostic for tolerances
    cond_SJ: float = float("nan")   # cond(Omega A_J) over occupied slots: diagnostic

    def min_margin(self):
        """Smallest |U - p| over the draws whose outcome was not forced."""
        ms = [abs(d.U - d.p) for d in self.decisions if 0.0 < d.p < 1.0]
        return min(ms) if ms else float("inf")


class OnlineRID:
    """Alg. 3 with Alg. 4 coefficients and the Alg. 8 error estimate."""

    def __init__(self, cfg: Config, n_max: int | None = None):
        self.cfg = cfg
        self.fill_mult = fill_factor(cfg)
        cap = n_max or 1024
        self.S = np.zeros((cfg.ell, cap))
        self.colsq = np.zeros(cap)
        self.SST = np.zeros((cfg.ell, cfg.ell))
        self.F = 0.0
        self.n_obs = 0
        self.D = []                       # buffered (snapshot index, column)
        self.J = np.full(cfg.t, -1, dtype=np.int64)
        self.J_prev = self.J.copy()
        self.tau_old = np.ones(cfg.t)
        self.C = None                     # m x t basis columns (data dtype)
        self.G = np.zeros((cfg.t, cfg.t))
        self.P = np.zeros((cfg.t, 0))
        self.u = 0
        self.records: list[UpdateRecord] = []

    # -- ingest ------------------------------------------------------------
    def _grow(self, need):
        cap = self.S.shape[1]
        if need <= cap:
            return
        new = max(need, 2 * cap)
        S = np.zeros((self.cfg.ell, new)); S[:, :cap] = self.S; self.S = S
        c = np.zeros(new); c[:cap] = self.colsq; self.colsq = c

    def push(self, cols):
        """Push snapshots given as the columns of an (m x b) array."""
        cols = np.asarray(cols)
        if cols.ndim == 1:
            cols = cols[:, None]
        cfg = self.cfg
        if cols.shape[0] != cfg.m:
            raise ValueError("snapshot length differs from m")
        if not np.all(np.isfinite(cols)):
            raise FloatingPointError("non-finite snapshot value")
        if self.C is None:
            self.C = np.zeros((cfg.m, cfg.t), dtype=cols.dtype)
        Sb, sq = sketch_columns(cols, cfg.omega_seed, cfg.ell, cfg.operand, cfg.row_chunk, cfg.workers)
        self._grow(self.n_obs + cols.shape[1])
        for jj in range(cols.shape[1]):
            j = self.n_obs
            s = Sb[:, jj]
            self.S[:, j] = s
            self.colsq[j] = sq[jj]
            self.SST += np.outer(s, s)
            self.F += sq[jj]
            self.D.append((j, cols[:, jj]))
            self.n_obs += 1
            if len(self.D) == cfg.t:
                self._update()

    def finalize(self):
        """Run the last update over a partially filled buffer."""
        if self.D:
            self._update()

    # -- one update (Alg. 3 steps 16-32) -----------------------------------
    def _update(self):
        cfg = self.cfg
        t = cfg.t
        rec = UpdateRecord(u=self.u, n_obs=self.n_obs, count=len(self.D), F=self.F)
        d_idx = [j for j, _ in self.D]
        S = self.S[:, :self.n_obs]
        filled = np.zeros(t, dtype=bool)
        J_before = self.J.copy()
        if self.F > 0.0:
            sk2, lam, mu = ridge_lambda(self.SST, self.F, cfg.k, cfg.ell, cfg.ridge_floor)
            rec.sk2, rec.lam = sk2, lam
            rec.kappa = float((mu[0] + cfg.ell * lam) / (max(mu[-1], 0.0) + cfg.ell * lam))
            occ = self.J >= 0
            tau_C = np.full(t, np.nan)
            if occ.any():
                tau_C[occ] = np.minimum(self.tau_old[occ], ridge_scores(self.SST, lam, cfg.ell, S[:, self.J[occ]]))
            tau_D = ridge_scores(self.SST, lam, cfg.ell, S[:, d_idx])
            J, tau_old, filled, decisions = select_slots(
                self.u, self.J, self.tau_old, tau_C, tau_D, d_idx, self.fill_mult, cfg.select_seed)
            rec.tau_C, rec.tau_D, rec.decisions = tau_C, tau_D, decisions
            rec.n_pruned = int(np.sum((J_before >= 0) & (J != J_before)))
            self.J, self.tau_old = J, tau_old
        else:
            rec.skipped = True
        rec.filled = filled
        rec.n_filled = int(filled.sum())
        # basis columns C (Alg. 3 fill step sets c_i = d_r; emptied slots are zero)
        C_prev = self.C.copy() if cfg.coeff == "best4" else None
        cols_by_idx = {j: col for j, col in self.D}
        for i in range(t):
            if filled[i]:
                self.C[:, i] = cols_by_idx[self.J[i]]
            elif self.J[i] < 0:
                self.C[:, i] = 0
        self.G = basis_gram(self.C, self.J)
        P4 = coeff_alg4(S, self.J)
        SJ = np.zeros((cfg.ell, t))
        occ = self.J >= 0
        SJ[:, occ] = S[:, self.J[occ]]
        if occ.any():
            sv = np.linalg.svd(SJ[:, occ], compute_uv=False)
            rec.cond_SJ = float(sv[0] / sv[-1]) if sv[-1] > 0 else float("inf")
        if cfg.coeff == "best4":
            # Alg. 3's coefficient steps: Algs. 4-7 each give P_q, NA-Hutch++
            # estimates its error, the smallest estimate wins (ties: lowest q).
            # Algs. 6 and 7 update the previous update's P, which covers the
            # columns observed up to that update; the columns observed since
            # take the Alg. 4 coefficients.
            n_prev = self.P.shape[1]
            P5 = coeff_alg5(S, self.J, self.G, cfg.ell)
            P6, P7 = P4.copy(), P4.copy()
            if n_prev:
                P6[:, :n_prev] = coeff_alg6(S, self.J, self.J_prev, self.P)
                T = alg7_transform(self.C, self.J, C_prev, self.J_prev)
                P7[:, :n_prev] = coeff_alg7(T, self.P)
            cands = [P4, P5, P6, P7]
            hs = [nahutchpp(S, SJ, Pq, self.G, self.F, cfg.n1, cfg.n2) for Pq in cands]
            rec.e2_q = [h["E2"] for h in hs]
            best = int(np.argmin(rec.e2_q))
            rec.q_star = 4 + best
            self.P = cands[best]
            rec.hutch = hs[best]
        else:
            self.P = P4
            rec.hutch = nahutchpp(S, SJ, self.P, self.G, self.F, cfg.n1, cfg.n2)
        rec.J = self.J.copy()
        self.records.append(rec)
        self.J_prev = self.J.copy()
        self.D = []
        self.u += 1


def basis_gram(C, J, row_chunk=1 << 18):
    """G = A_J^T A_J in binary64 (zero rows and columns for empty slots)."""
    t = C.shape[1]
    G = np.zeros((t, t))
    occ = np.flatnonzero(np.asarray(J) >= 0)
    if occ.size == 0:
        return G
    for i0 in range(0, C.shape[0], row_chunk):
        blk = C[i0:i0 + row_chunk, occ].astype(np.float64)
        G[np.ix_(occ, occ)] += blk.T @ blk
    return G
