"""Seeded synthetic snapshot streams (inputs only; no step of the method).

Both the oracle and the HIP path consume the bytes these functions produce, so
the same module serves both sides.  The paper's datasets (turbulent channel
flow, ignition, NSTX gas-puff images; Sec. 4) are not available; these streams
take their shapes and structure instead.  Every generator returns the snapshot
matrix column-major as a C-contiguous (n, m) array: row j of the result is
snapshot j (a contiguous column of A).

* ``sines``      - sum of 20 travelling sines with decaying amplitudes plus
                   1e-6 noise (a toy stream whose clean part has rank <= 40).
* ``lowrank``    - U diag(sigma) V^T with sigma_i = exp(-i/10) plus relative
                   1e-5 noise (a generic low-rank stream).
* ``channel``    - four fields (u, v, w, p) on an x-y-z grid, each a sum of
                   travelling Fourier modes with k^(-5/3) amplitudes and a
                   tanh wall profile (stands in for channel flow).
* ``blobs``      - advected Gaussian blobs with 1% noise on a 2D frame (stands
                   in for gas-puff images).
"""
from __future__ import annotations

import math

import numpy as np

DATA_SEED_BASE = 24051607600


def data_seed(cfg_index):
    return DATA_SEED_BASE + int(cfg_index)


# --------------------------------------------------------------------------
# toy: sum of travelling sines
# --------------------------------------------------------------------------

def sines(m, n, seed, dtype=np.float64, noise=1e-6, modes=20):
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi, modes)
    x = np.arange(m, dtype=np.float64) / m
    i = np.arange(1, modes + 1, dtype=np.float64)
    amp = np.exp(-i / 3.0)
    tt = np.arange(n, dtype=np.float64)
    # snapshot t: sum_i amp_i sin(2 pi i x + 0.05 i t + phi_i)
    ph = 0.05 * i[None, :] * tt[:, None] + phi[None, :]            # (n, modes)
    base_s = np.sin(2.0 * math.pi * i[:, None] * x[None, :])        # (modes, m)
    base_c = np.cos(2.0 * math.pi * i[:, None] * x[None, :])
    out = (np.cos(ph) * amp) @ base_s + (np.sin(ph) * amp) @ base_c  # (n, m)
    out += noise * rng.standard_normal((n, m))
    return np.ascontiguousarray(out.astype(dtype))


# --------------------------------------------------------------------------
# generic low rank
# --------------------------------------------------------------------------

def lowrank(m, n, seed, rank=200, dtype=np.float32, rel_noise=1e-5, decay=10.0):
    rng = np.random.default_rng(seed)
    r = min(rank, m, n)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    sig = np.exp(-np.arange(1, r + 1) / decay)
    clean = (V * sig) @ U.T                                        # (n, m)
    rms = math.sqrt(float(np.mean(clean * clean)))
    out = clean + rel_noise * rms * rng.standard_normal((n, m))
    return np.ascontiguousarray(out.astype(dtype))


# --------------------------------------------------------------------------
# channel-flow-shaped modes
# --------------------------------------------------------------------------

def channel_modes(seed, n_modes=300, kmax=24, fields=4):
    """Random mode table of the channel stream (small arrays)."""
    rng = np.random.default_rng(seed)
    pairs = [(kx, kz) for kx in range(0, kmax + 1) for kz in range(-kmax, kmax + 1)
             if 1.0 <= math.hypot(kx, kz) <= kmax]
    pick = rng.integers(0, len(pairs), n_modes)
    kx = np.array([pairs[p][0] for p in pick], dtype=np.float64)
    kz = np.array([pairs[p][1] for p in pick], dtype=np.float64)
    kappa = np.hypot(kx, kz)
    amp = kappa ** (-5.0 / 3.0)
    c = rng.uniform(0.6, 1.0, n_modes)
    omega = 0.05 * kx * c + 0.01 * kz
    beta = rng.uniform(4.0, 16.0, n_modes)
    r = rng.uniform(0.5, 1.5, (fields, n_modes))
    ph = rng.uniform(0.0, 2.0 * math.pi, (fields, n_modes))
    fscale = np.ones(fields)
    if fields >= 4:
        fscale[3] = 0.5
    return dict(kx=kx, kz=kz, amp=amp, omega=omega, beta=beta, r=r, phase=ph, fscale=fscale)


def channel_grid(nx, ny, nz):
    x = np.arange(nx) / nx            # x / (8 pi), periodic
    z = np.arange(nz) / nz            # z / (3 pi), periodic
    y = -np.cos(math.pi * np.arange(ny) / (ny - 1))
    return x, y, z


def channel_spatial_rows(modes, grid, field, rows):
    """Spatial factor B (len(rows) x (2 * n_modes + 1)) for one field, at the
    flattened grid positions ``rows`` (x fastest, then z, then y):
    A(:, t) = B @ T(:, t) with T = [cos(w t); sin(w t); 1]."""
    nx, ny, nz = grid
    x, y, z = channel_grid(nx, ny, nz)
    ix = rows % nx
    iz = (rows // nx) % nz
    iy = rows // (nx * nz)
    th = 2.0 * math.pi * (np.outer(x[ix], modes["kx"]) + np.outer(z[iz], modes["kz"])) + modes["phase"][field][None, :]
    g = np.tanh(np.outer(1.0 - np.abs(y[iy]), modes["beta"]))
    w = (modes["amp"] * modes["r"][field] * modes["fscale"][field])[None, :] * g
    # sin(th - w t) = sin(th) cos(w t) - cos(th) sin(w t)
    mean = np.tanh(8.0 * (1.0 - np.abs(y[iy]))) if field == 0 else np.zeros(len(rows))
    return np.concatenate([w * np.sin(th), -w * np.cos(th), mean[:, None]], axis=1)


def channel_temporal(modes, n, t0=0):
    tt = np.arange(t0, t0 + n, dtype=np.float64)
    wt = np.outer(modes["omega"], tt)
    return np.concatenate([np.cos(wt), np.sin(wt), np.ones((1, n))], axis=0)


def channel(nx, ny, nz, n, seed, fields=4, n_modes=300, dtype=np.float32):
    """Channel stream on a small grid, computed on the host."""
    modes = channel_modes(seed, n_modes=n_modes, fields=fields)
    npts = nx * ny * nz
    T = channel_temporal(modes, n)
    out = np.empty((n, fields * npts), dtype=dtype)
    rows = np.arange(npts)
    for f in range(fields):
        B = channel_spatial_rows(modes, (nx, ny, nz), f, rows)
        out[:, f * npts:(f + 1) * npts] = (B @ T).T.astype(dtype)
    return out


# --------------------------------------------------------------------------
# image stream: advected Gaussian blobs
# --------------------------------------------------------------------------

def blobs(h, w, n, seed, n_blobs=6, rel_noise=0.01, dtype=np.float32):
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.5, 1.5, n_blobs)
    wid = rng.uniform(0.03, 0.1, n_blobs) * min(h, w)
    vel = rng.uniform(-1.0, 1.0, (n_blobs, 2)) * 0.002 * max(h, w)
    pos0 = rng.uniform(0.0, 1.0, (n_blobs, 2)) * np.array([h, w])
    yy, xx = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    out = np.empty((n, h * w), dtype=dtype)
    for t in range(n):
        fr = np.zeros((h, w))
        for b in range(n_blobs):
            cy, cx = pos0[b] + vel[b] * t
            dy = (yy - cy + h / 2) % h - h / 2
            dx = (xx - cx + w / 2) % w - w / 2
            fr += amp[b] * np.exp(-(dy * dy + dx * dx) / (2.0 * wid[b] ** 2))
        rms = math.sqrt(float(np.mean(fr * fr)))
        fr += rel_noise * rms * rng.standard_normal((h, w))
        out[t] = fr.reshape(-1)
    return out


def blobs_torch(h, w, n, seed, n_blobs=6, rel_noise=0.01, device="cuda:0", ld=None):
    """The blob stream generated on a device with torch (same recipe as
    ``blobs``; blob parameters from the same numpy draws, the noise from a
    seeded torch generator, so the noise differs from ``blobs``).  Returns an
    (n, ld) binary32 tensor whose [:, :h w] view holds the frames; ld defaults
    to h w rounded up to 16 elements."""
    import torch
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.5, 1.5, n_blobs)
    wid = rng.uniform(0.03, 0.1, n_blobs) * min(h, w)
    vel = rng.uniform(-1.0, 1.0, (n_blobs, 2)) * 0.002 * max(h, w)
    pos0 = rng.uniform(0.0, 1.0, (n_blobs, 2)) * np.array([h, w])
    dev = torch.device(device)
    m = h * w
    ld = ld or (m + 15) // 16 * 16
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed) % (1 << 63))
    yy = torch.arange(h, device=dev, dtype=torch.float32)[None, :, None]
    xx = torch.arange(w, device=dev, dtype=torch.float32)[None, None, :]
    out = torch.zeros((n, ld), dtype=torch.float32, device=dev)
    chunk = max(1, (1 << 25) // max(m, 1))  # frames per chunk (~128 MB of binary32)
    for t0 in range(0, n, chunk):
        t = torch.arange(t0, min(n, t0 + chunk), device=dev, dtype=torch.float64)
        fr = torch.zeros((t.numel(), h, w), dtype=torch.float32, device=dev)
        for b in range(n_blobs):
            cy = (pos0[b, 0] + vel[b, 0] * t).to(torch.float32)[:, None, None]
            cx = (pos0[b, 1] + vel[b, 1] * t).to(torch.float32)[:, None, None]
            dy = torch.remainder(yy - cy + h / 2, h) - h / 2
            dx = torch.remainder(xx - cx + w / 2, w) - w / 2
            fr += float(amp[b]) * torch.exp(-(dy * dy + dx * dx) / float(2.0 * wid[b] ** 2))
        rms = torch.sqrt(torch.mean(fr * fr, dim=(1, 2), keepdim=True))
        fr += rel_noise * rms * torch.randn(fr.shape, generator=g, device=dev, dtype=torch.float32)
        out[t0:t0 + t.numel(), :m] = fr.reshape(t.numel(), m)
    return out


def batch_frame_shapes(ns, seed, lo=1e4, hi=1e6):
    """Frame sizes of a batch of image streams: m log-uniform in [lo, hi],
    frames h x w with h = round(sqrt(0.8 m)) and w = round(m / h) (the 4:5
    aspect of the gas-puff images), m := h w."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(ns):
        m = int(round(10.0 ** rng.uniform(math.log10(lo), math.log10(hi))))
        h = max(1, int(round(math.sqrt(0.8 * m))))
        w = max(1, int(round(m / h)))
        out.append((h, w))
    return out


def channel_torch(nx, ny, nz, n, seed, fields=4, n_modes=300, device="cuda:0", rows_per_chunk=1 << 20,
                  ld=None):
    """The channel stream generated on a device with torch (same mode table and
    recipe as ``channel``; evaluated in binary64, stored as binary32).  Returns
    an (n, ld) tensor whose [:, :m] view holds the snapshots; ld defaults to m
    rounded up to 64 elements."""
    import torch
    modes = channel_modes(seed, n_modes=n_modes, fields=fields)
    npts = nx * ny * nz
    m = fields * npts
    ld = ld or (m + 63) // 64 * 64
    dev = torch.device(device)
    T = torch.tensor(channel_temporal(modes, n), dtype=torch.float64, device=dev).to(torch.float32)
    x, y, z = channel_grid(nx, ny, nz)
    xt = torch.tensor(x, dtype=torch.float64, device=dev)
    yt = torch.tensor(y, dtype=torch.float64, device=dev)
    zt = torch.tensor(z, dtype=torch.float64, device=dev)
    kx = torch.tensor(modes["kx"], dtype=torch.float64, device=dev)
    kz = torch.tensor(modes["kz"], dtype=torch.float64, device=dev)
    beta = torch.tensor(modes["beta"], dtype=torch.float64, device=dev)
    out = torch.empty((n, ld), dtype=torch.float32, device=dev)
    for f in range(fields):
        w0 = torch.tensor(modes["amp"] * modes["r"][f] * modes["fscale"][f], dtype=torch.float64, device=dev)
        ph = torch.tensor(modes["phase"][f], dtype=torch.float64, device=dev)
        for r0 in range(0, npts, rows_per_chunk):
            r1 = min(npts, r0 + rows_per_chunk)
            rows = torch.arange(r0, r1, device=dev)
            ix = rows % nx
            iz = (rows // nx) % nz
            iy = rows // (nx * nz)
            th = 2.0 * math.pi * (torch.outer(xt[ix], kx) + torch.outer(zt[iz], kz)) + ph[None, :]
            ay = 1.0 - torch.abs(yt[iy])
            w = w0[None, :] * torch.tanh(torch.outer(ay, beta))
            mean = torch.tanh(8.0 * ay) if f == 0 else torch.zeros_like(ay)
            B = torch.cat([w * torch.sin(th), -w * torch.cos(th), mean[:, None]], dim=1).to(torch.float32)
            del th, w
            out[:, f * npts + r0:f * npts + r1] = (B @ T).T
            del B
    return out
