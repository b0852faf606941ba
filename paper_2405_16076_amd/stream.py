"""Python binding of the streaming randomized ID (include/rid.h).

Argument marshalling only: every step runs in the HIP library.  Snapshot
batches are CUDA tensors of shape (b, m) (each row one contiguous snapshot,
i.e. b columns of A); results come back as numpy arrays or CUDA tensors.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

_DTYPE = {torch.float32: L.RID_F32, torch.float64: L.RID_F64}
PREC = {"f64": L.RID_SKETCH_F64, "f32": L.RID_SKETCH_F32, "bf16": L.RID_SKETCH_BF16, "fp8": L.RID_SKETCH_FP8}


@dataclass
class StreamConfig:
    m: int
    ell: int
    k: int
    t: int
    n_max: int
    dtype: torch.dtype = torch.float32
    sketch: str = "f32"
    omega_seed: int = 1
    select_seed: int = 2
    delta: float = 0.05
    eps: float = 0.5
    c_sample: float = 1.0
    ridge_floor: float = 1e-8
    hutch_n1: int = 0
    hutch_n2: int = 0
    lookahead: int = 0
    tile: str = "auto"   # bf16 sketch work split: auto, narrow or wide
    coeff: str = "alg4"  # "alg4" or "best4" (the best of Algs. 4-7 at every update)
    gram: str = "auto"   # basis Gram of binary32 data: "auto", "exact" (binary64 products) or "split"

    def to_c(self):
        c = L.rid_config()
        L.check(L.lib().rid_config_default(C.byref(c)))
        c.m, c.ell, c.k, c.t, c.n_max = self.m, self.ell, self.k, self.t, self.n_max
        c.data_dtype = _DTYPE[self.dtype]
        c.sketch_prec = PREC[self.sketch]
        c.omega_seed, c.select_seed = self.omega_seed, self.select_seed
        c.delta, c.eps, c.c_sample, c.ridge_floor = self.delta, self.eps, self.c_sample, self.ridge_floor
        c.hutch_n1, c.hutch_n2, c.lookahead = self.hutch_n1, self.hutch_n2, self.lookahead
        c.sketch_tile = {"auto": L.RID_TILE_AUTO, "narrow": L.RID_TILE_NARROW, "wide": L.RID_TILE_WIDE}[self.tile]
        c.coeff_mode = {"alg4": L.RID_COEFF_ALG4, "best4": L.RID_COEFF_BEST4}[self.coeff]
        c.gram_mode = {"auto": L.RID_GRAM_AUTO, "exact": L.RID_GRAM_EXACT, "split": L.RID_GRAM_SPLIT}[self.gram]
        return c


def _stream_handle(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class OnlineRID:
    """One streaming randomized ID on one GPU (Alg. 3 with Alg. 4 and Alg. 8)."""

    def __init__(self, cfg: StreamConfig, device="cuda:0", _member=None):
        self.cfg = cfg
        self.device = torch.device(device)
        self._keep = []  # borrowed batches kept alive until release
        if _member is not None:  # a member of a StreamBatch (owned by it)
            self._h = _member
            self._owned = False
            return
        self._h = C.c_void_p()
        self._owned = True
        ccfg = cfg.to_c()
        with torch.cuda.device(self.device):
            L.check(L.lib().rid_init_stream(C.byref(ccfg), _stream_handle(self.device), C.byref(self._h)))

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if self._h and self._owned:
            L.lib().rid_destroy(self._h)
        self._h = C.c_void_p()
        self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        L.check(st, self._h)

    # -- ingest --------------------------------------------------------------
    def push(self, cols: torch.Tensor, borrow: bool = False):
        """Push a (b, m) CUDA tensor of snapshots (row j = snapshot j)."""
        if cols.dim() == 1:
            cols = cols.unsqueeze(0)
        if cols.device != self.device or cols.dtype != self.cfg.dtype or cols.shape[1] != self.cfg.m:
            raise ValueError("snapshots must be a (b, m) tensor of the stream's dtype on its device")
        if cols.stride(1) != 1:
            raise ValueError("each snapshot must be contiguous")
        flags = L.RID_BORROW if borrow else L.RID_COPY
        self._check(L.lib().rid_push_snapshots(self._h, C.c_void_p(cols.data_ptr()), cols.stride(0),
                                                cols.shape[0], flags))
        if borrow:
            self._keep.append(cols)

    def flush(self):
        self._check(L.lib().rid_flush(self._h))

    def finalize(self):
        self._check(L.lib().rid_finalize(self._h))

    def reset(self):
        self._check(L.lib().rid_reset(self._h))
        self._keep = []

    # -- results -------------------------------------------------------------
    def select(self):
        J = np.empty(self.cfg.t, dtype=np.int64)
        t = C.c_int32()
        self._check(L.lib().rid_select(self._h, J.ctypes.data_as(C.POINTER(C.c_int64)), self.cfg.t, C.byref(t)))
        return J

    def coefficients(self, device=False):
        info = self.info()
        cap = max(int(info.n_pushed), 1)
        n = C.c_int64()
        if device:
            P = torch.empty((cap, self.cfg.t), dtype=torch.float64, device=self.device)
            self._check(L.lib().rid_coefficients(self._h, C.c_void_p(P.data_ptr()), self.cfg.t, cap,
                                                 C.byref(n), L.RID_DEVICE))
            return P[:n.value].T
        P = np.zeros((cap, self.cfg.t), dtype=np.float64)
        self._check(L.lib().rid_coefficients(self._h, P.ctypes.data_as(C.c_void_p), self.cfg.t, cap,
                                             C.byref(n), L.RID_HOST))
        return np.ascontiguousarray(P[:n.value].T)

    def error_estimate(self):
        e = L.rid_error()
        self._check(L.lib().rid_error_estimate(self._h, C.byref(e)))
        return dict(E2=e.E2, E=e.E_abs, rel=e.rel, F=e.F, n_obs=e.n_obs, update=e.update)

    def reconstruct(self, j0, c):
        out = torch.empty((c, self.cfg.m), dtype=self.cfg.dtype, device=self.device)
        self._check(L.lib().rid_reconstruct(self._h, j0, c, C.c_void_p(out.data_ptr()), self.cfg.m))
        return out

    def info(self):
        i = L.rid_info()
        self._check(L.lib().rid_get_info(self._h, C.byref(i)))
        return i

    def coeff_choice(self, u):
        """(E^2 of Algs. 4, 5, 6, 7, the kept algorithm) of update u (best4 mode)."""
        e2 = np.zeros(4, dtype=np.float64)
        q = C.c_int32()
        self._check(L.lib().rid_get_coeff_choice(self._h, u, e2.ctypes.data_as(C.c_void_p), C.byref(q)))
        return e2, q.value

    def update(self, u):
        rec = L.rid_update()
        t = self.cfg.t
        J = np.empty(t, dtype=np.int64)
        tc = np.empty(t, dtype=np.float64)
        td = np.empty(t, dtype=np.float64)
        self._check(L.lib().rid_get_update(self._h, u, C.byref(rec), J.ctypes.data_as(C.c_void_p),
                                           tc.ctypes.data_as(C.c_void_p), td.ctypes.data_as(C.c_void_p)))
        d = {f: getattr(rec, f) for f, _ in L.rid_update._fields_}
        d["J"] = J
        d["tau_C"] = tc
        d["tau_D"] = td[:rec.count].copy()
        return d

    def profile_enable(self, on=True):
        self._check(L.lib().rid_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        p = L.rid_profile()
        self._check(L.lib().rid_profile_read(self._h, C.byref(p)))
        return {f: getattr(p, f) for f, _ in L.rid_profile._fields_}

    def debug_state(self):
        info = self.info()
        n = int(info.n_pushed)
        S = np.zeros((max(n, 1), self.cfg.ell), dtype=np.float64)
        q = np.zeros(max(n, 1), dtype=np.float64)
        G = np.zeros((self.cfg.t, self.cfg.t), dtype=np.float64)
        nc = C.c_int64()
        self._check(L.lib().rid_debug_state(self._h, S.ctypes.data_as(C.c_void_p), self.cfg.ell, max(n, 1),
                                            C.byref(nc), q.ctypes.data_as(C.c_void_p),
                                            G.ctypes.data_as(C.c_void_p)))
        k = nc.value
        return np.ascontiguousarray(S[:k].T), q[:k].copy(), G.T.copy()


def omega_block(prec, seed, ell, i0, count, device="cuda:0"):
    """Omega(0:ell, i0:i0+count) as the sketch form `prec` evaluates it."""
    dt = torch.float64 if prec == "f64" else torch.float32
    out = torch.empty((count, ell), dtype=dt, device=device)
    with torch.cuda.device(torch.device(device)):
        L.check(L.lib().rid_omega_block(PREC[prec], seed, ell, i0, count, C.c_void_p(out.data_ptr()), ell,
                                        _stream_handle(torch.device(device))))
    return out.T


def _sketch_args(X, ell):
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a (b, m) tensor with unit element stride")
    if X.dtype not in (torch.float32, torch.float64):
        raise ValueError("X must be float32 or float64")
    b, m = X.shape
    S = torch.empty((b, ell), dtype=torch.float64, device=X.device)
    colsq = torch.empty(b, dtype=torch.float64, device=X.device)
    flag = torch.empty(1, dtype=torch.int32, device=X.device)
    return b, m, S, colsq, flag


def sketch_columns(X, ell, omega_seed, sketch="bf16"):
    """S = Omega A (l x b, binary64), ||a_j||^2 and the non-finite flag for the
    b snapshots held in the rows of X (b, m) (rid_sketch_columns)."""
    b, m, S, colsq, flag = _sketch_args(X, ell)
    with torch.cuda.device(X.device):
        L.check(L.lib().rid_sketch_columns(PREC[sketch], omega_seed, ell, m, C.c_void_p(X.data_ptr()), X.stride(0),
                                           b, C.c_void_p(S.data_ptr()), C.c_void_p(colsq.data_ptr()),
                                           C.c_void_p(flag.data_ptr()), _stream_handle(X.device)))
    return S.T, colsq, flag


def sketch_columns_noalloc(X, ell, omega_seed, sketch, S, colsq, flag):
    """rid_sketch_columns_noalloc into caller-provided outputs: S (b, l)
    binary64 (read as l x b column-major), colsq (b,) binary64, flag (1,)
    int32.  The library allocates nothing."""
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be a (b, m) tensor with unit element stride")
    b, m = X.shape
    if S.shape != (b, ell) or not S.is_contiguous() or S.dtype != torch.float64:
        raise ValueError("S must be a contiguous (b, l) float64 tensor")
    if colsq.shape != (b,) or colsq.dtype != torch.float64 or flag.dtype != torch.int32:
        raise ValueError("colsq must be (b,) float64 and flag int32")
    with torch.cuda.device(X.device):
        L.check(L.lib().rid_sketch_columns_noalloc(PREC[sketch], omega_seed, ell, m, C.c_void_p(X.data_ptr()),
                                                   X.stride(0), b, C.c_void_p(S.data_ptr()),
                                                   C.c_void_p(colsq.data_ptr()), C.c_void_p(flag.data_ptr()),
                                                   _stream_handle(X.device)))


class StreamBatch:
    """Many independent streams of uneven m advanced together: one persistent
    sketch launch per round over every member, batched update launches, the
    round captured into a HIP graph (rid_init_batch and friends)."""

    def __init__(self, cfgs, device="cuda:0", graph=True, tune=True):
        self.cfgs = list(cfgs)
        self.device = torch.device(device)
        self._b = C.c_void_p()
        arr = (L.rid_config * len(self.cfgs))(*[c.to_c() for c in self.cfgs])
        flags = (0 if graph else L.RID_BATCH_NO_GRAPH) | (0 if tune else L.RID_BATCH_NO_TUNE)
        with torch.cuda.device(self.device):
            L.check(L.lib().rid_init_batch(len(self.cfgs), arr, _stream_handle(self.device), flags,
                                           C.byref(self._b)), batch=None)
        self.members = []
        for i, c in enumerate(self.cfgs):
            h = C.c_void_p()
            self._check(L.lib().rid_batch_stream(self._b, i, C.byref(h)))
            self.members.append(OnlineRID(c, device, _member=h))
        self._keep = []

    def _check(self, st):
        L.check(st, batch=self._b)

    def close(self):
        if self._b:
            for mbr in self.members:
                mbr._h = C.c_void_p()
            L.lib().rid_destroy_batch(self._b)
            self._b = C.c_void_p()
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, cols, borrow=False):
        """cols: one (b_i, m_i) CUDA tensor (or None) per member."""
        ns = len(self.cfgs)
        if len(cols) != ns:
            raise ValueError("one tensor (or None) per member")
        ptrs = (C.c_void_p * ns)()
        lds = (C.c_int64 * ns)()
        bs = (C.c_int32 * ns)()
        for i, (x, c) in enumerate(zip(cols, self.cfgs)):
            if x is None or x.shape[0] == 0:
                ptrs[i], lds[i], bs[i] = None, c.m, 0
                continue
            if x.device != self.device or x.dtype != c.dtype or x.shape[1] != c.m or x.stride(1) != 1:
                raise ValueError(f"member {i}: snapshots must be a (b, m) tensor of its dtype, rows contiguous")
            ptrs[i], lds[i], bs[i] = x.data_ptr(), x.stride(0), x.shape[0]
        self._check(L.lib().rid_push_batch(self._b, ptrs, lds, bs, L.RID_BORROW if borrow else L.RID_COPY))
        if borrow:
            self._keep.append(list(cols))

    def finalize(self):
        self._check(L.lib().rid_finalize_batch(self._b))

    def reset(self):
        self._check(L.lib().rid_reset_batch(self._b))
        self._keep = []

    def profile_enable(self, on=True):
        self._check(L.lib().rid_batch_profile_enable(self._b, 1 if on else 0))

    def profile_read(self):
        p = L.rid_profile()
        self._check(L.lib().rid_batch_profile_read(self._b, C.byref(p)))
        d = {f: getattr(p, f) for f, _ in L.rid_profile._fields_}
        d["rounds"] = d.pop("updates")
        return d

    def tune_table(self):
        """[(slab_rows, tile, ms)] of the candidates the slab tuner timed."""
        out = []
        rows, wide, ms = C.c_int64(), C.c_int32(), C.c_double()
        while L.lib().rid_batch_tune_result(self._b, len(out), C.byref(rows), C.byref(wide), C.byref(ms)) == L.RID_OK:
            out.append((rows.value, "wide" if wide.value else "narrow", round(ms.value, 3)))
        return out

    def info(self):
        i = L.rid_batch_info()
        self._check(L.lib().rid_batch_get_info(self._b, C.byref(i)))
        return {f: getattr(i, f) for f, _ in L.rid_batch_info._fields_}
