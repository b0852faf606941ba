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
* ``ignition``   - ten species and a temperature on a 3D grid around a
                   wrinkled reaction front that moves at a randomised speed,
                   fields spanning ~1e7 in magnitude, each with 64 travelling
                   modes of i^-2 amplitude (stands in for the ignition data).

The ``*_torch`` variants generate on a GPU; ``ignition_torch`` and
``blobs_torch`` can write a window of time steps into a caller's buffer, so a
long stream can be produced round by round into a ring of borrowed columns.
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


def blobs_torch(h, w, n, seed, n_blobs=6, rel_noise=0.01, device="cuda:0", ld=None, t_start=0, out=None):
    """The blob stream generated on a device with torch (same recipe as
    ``blobs``; blob parameters from the same numpy draws, the noise from a
    seeded torch generator, so the noise differs from ``blobs``).  Returns an
    (n, ld) binary32 tensor whose [:, :h w] view holds frames t_start ..
    t_start + n - 1; ld defaults to h w rounded up to 16 elements.  With
    ``out`` (an (n, ld) binary32 tensor) the frames are written there.  The
    noise generator is seeded by (seed, t_start), so a window generated on its
    own equals the same window of a call that starts there."""
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
    g.manual_seed((int(seed) + 1000003 * int(t_start)) % (1 << 63))
    yy = torch.arange(h, device=dev, dtype=torch.float32)[None, :, None]
    xx = torch.arange(w, device=dev, dtype=torch.float32)[None, None, :]
    if out is None:
        out = torch.zeros((n, ld), dtype=torch.float32, device=dev)
    chunk = max(1, (1 << 25) // max(m, 1))  # frames per chunk (~128 MB of binary32)
    for t0 in range(0, n, chunk):
        t = torch.arange(t_start + t0, t_start + min(n, t0 + chunk), device=dev, dtype=torch.float64)
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


# --------------------------------------------------------------------------
# generic low rank, on a device
# --------------------------------------------------------------------------

def lowrank_torch(m, n, seed, rank=200, rel_noise=1e-5, decay=10.0, device="cuda:0", ld=None):
    """U diag(sigma) V^T + relative noise generated on a device: U (m x r) and
    V (n x r) the Q factors of seeded Gaussians, sigma_i = exp(-i / decay),
    noise rel_noise * rms(clean) * N(0, 1).  Returns an (n, ld) binary32
    tensor whose [:, :m] view holds the snapshots (ld = m rounded up to 64)."""
    import torch
    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed) % (1 << 63))
    r = min(rank, m, n)
    ld = ld or (m + 63) // 64 * 64
    U, _ = torch.linalg.qr(torch.randn((m, r), generator=g, device=dev, dtype=torch.float64))
    V, _ = torch.linalg.qr(torch.randn((n, r), generator=g, device=dev, dtype=torch.float64))
    sig = torch.exp(-torch.arange(1, r + 1, device=dev, dtype=torch.float64) / decay)
    out = torch.empty((n, ld), dtype=torch.float32, device=dev)
    Vs = (V * sig).contiguous()
    rows = max(1, (1 << 28) // max(m, 1))
    sq = 0.0
    for j0 in range(0, n, rows):
        blk = Vs[j0:j0 + rows] @ U.T.contiguous()
        sq += float(torch.sum(blk * blk))
        out[j0:j0 + blk.shape[0], :m] = blk.to(torch.float32)
        del blk
    rms = math.sqrt(sq / (float(m) * n))
    for j0 in range(0, n, rows):
        j1 = min(n, j0 + rows)
        out[j0:j1, :m] += (rel_noise * rms) * torch.randn((j1 - j0, m), generator=g, device=dev,
                                                          dtype=torch.float32)
    del U, V, Vs
    return out


# --------------------------------------------------------------------------
# ignition-shaped stream: ten species and a temperature around a moving,
# wrinkled reaction front on a 3D grid
# --------------------------------------------------------------------------

IGNITION_FIELDS = 11


def ignition_params(seed, n_total, n_modes=64):
    """Mode table and front trajectory of the ignition stream (numpy draws).

    Front position s(t) = 0.1 + sum_{tau < t} vbar (1 + 0.5 xi_tau) with
    xi ~ U(-1, 1) and vbar = 0.8 / n_total; wrinkle amplitudes i^-2 (i = 1..8)
    with phases psi, chi; species scales log-spaced from 1 down to 1e-4 and
    front widths 0.01 (1 + j / 10); per field 64 travelling modes with integer
    wave vectors (|k_d| <= 6), speeds omega ~ U(0, 0.05) per step and phases
    per field."""
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, n_total)
    vbar = 0.8 / n_total
    front = 0.1 + np.concatenate([[0.0], np.cumsum(vbar * (1.0 + 0.5 * xi))[:-1]])
    psi = rng.uniform(0.0, 2.0 * math.pi, 8)
    chi = rng.uniform(0.0, 2.0 * math.pi, 8)
    kvec = rng.integers(-6, 7, size=(n_modes, 3))
    kvec[np.all(kvec == 0, axis=1)] = (1, 0, 0)
    omega = rng.uniform(0.0, 0.05, n_modes)
    phase = rng.uniform(0.0, 2.0 * math.pi, (IGNITION_FIELDS, n_modes))
    scale = 10.0 ** (-4.0 * np.arange(10) / 9.0)
    width = 0.01 * (1.0 + np.arange(10) / 10.0)
    return dict(front=front, psi=psi, chi=chi, kvec=kvec, omega=omega, phase=phase, scale=scale, width=width)


class IgnitionStream:
    """Generator of the ignition stream on a device, a window of time steps at
    a time.  Grid (n1, n2, n3) of cell centres on [0, 1]^3, x1 fastest; field
    f occupies rows [f npts, (f + 1) npts) of a snapshot (T first, then the
    ten species).  Fields:

    * T = 300 + 1700 (1 + tanh((x_f - x1) / 0.01)) / 2, x_f = s(t) +
      0.02 sum_{i=1..8} i^-2 sin(2 pi i x2 + psi_i) cos(2 pi i x3 + chi_i);
    * species 0-2 (reactants) scale (1 - tanh((x_f - x1) / w)) / 2, 3-4
      (products) scale (1 + tanh(...)) / 2, 5-9 (intermediates)
      scale sech^2((x_f - x1) / w);
    * every field adds 0.05 scale_f sum_{i=1..64} i^-2 sin(2 pi k_i . x +
      omega_i t + phi_{i,f}) (scale 1700 for T), evaluated as the product of
      the spatial sin / cos table (npts x 128, shared by the fields) with the
      per-field temporal coefficients.
    Evaluated in binary32."""

    def __init__(self, n1, n2, n3, n_total, seed, device="cuda:0", n_modes=64):
        import torch
        self.shape = (n1, n2, n3)
        self.npts = n1 * n2 * n3
        self.m = IGNITION_FIELDS * self.npts
        self.n_total = n_total
        self.p = ignition_params(seed, n_total, n_modes)
        self.dev = torch.device(device)
        f32 = torch.float32
        idx = torch.arange(self.npts, device=self.dev)
        i1 = idx % n1
        i2 = (idx // n1) % n2
        i3 = idx // (n1 * n2)
        self.x1 = ((i1.to(torch.float64) + 0.5) / n1).to(f32)
        x2 = (i2.to(torch.float64) + 0.5) / n2
        x3 = (i3.to(torch.float64) + 0.5) / n3
        wr = torch.zeros(self.npts, dtype=torch.float64, device=self.dev)
        for i in range(1, 9):
            wr += (i ** -2.0) * torch.sin(2 * math.pi * i * x2 + self.p["psi"][i - 1]) * \
                torch.cos(2 * math.pi * i * x3 + self.p["chi"][i - 1])
        self.wrinkle = (0.02 * wr).to(f32)
        k = torch.tensor(self.p["kvec"], dtype=torch.float64, device=self.dev)
        x1d = (i1.to(torch.float64) + 0.5) / n1
        th = 2 * math.pi * (torch.outer(x1d, k[:, 0]) + torch.outer(x2, k[:, 1]) + torch.outer(x3, k[:, 2]))
        amp = torch.tensor(np.arange(1, n_modes + 1, dtype=np.float64) ** -2.0, device=self.dev)
        # sin(th + a) = sin(th) cos(a) + cos(th) sin(a)
        self.table = torch.cat([torch.sin(th) * amp, torch.cos(th) * amp], dim=1).to(f32)   # (npts, 128)
        del th, x2, x3, wr, k, x1d, idx, i1, i2, i3
        self.field_scale = [1700.0] + list(self.p["scale"])

    def generate(self, t0, b, out):
        """Writes snapshots t0 .. t0 + b - 1 into rows 0 .. b - 1 of out
        ((>= b, ld >= m) binary32 tensor)."""
        import torch
        p = self.p
        npts = self.npts
        f32 = torch.float32
        tt = torch.arange(t0, t0 + b, device=self.dev, dtype=torch.float64)
        front = torch.tensor(p["front"][t0:t0 + b], device=self.dev, dtype=torch.float64).to(f32)
        om = torch.tensor(p["omega"], device=self.dev, dtype=torch.float64)
        for f in range(IGNITION_FIELDS):
            a = torch.outer(tt, om) + torch.tensor(p["phase"][f], device=self.dev)[None, :]   # (b, modes)
            coef = (0.05 * self.field_scale[f]) * torch.cat([torch.cos(a), torch.sin(a)], dim=1)
            dst = out[:b, f * npts:(f + 1) * npts]
            torch.matmul(coef.to(f32), self.table.T, out=dst)
            d = front[:, None] + self.wrinkle[None, :] - self.x1[None, :]      # x_f - x1, (b, npts)
            if f == 0:
                dst += 300.0 + 850.0 * (1.0 + torch.tanh(d / 0.01))
            else:
                j = f - 1
                sc, wd = float(p["scale"][j]), float(p["width"][j])
                if j < 3:
                    dst += (0.5 * sc) * (1.0 - torch.tanh(d / wd))
                elif j < 5:
                    dst += (0.5 * sc) * (1.0 + torch.tanh(d / wd))
                else:
                    dst += sc / torch.cosh(d / wd) ** 2
            del d, a, coef
        return out
