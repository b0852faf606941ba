"""The Gaussian test matrix Omega of the oracle (test infrastructure only).

The paper draws Omega (l x m) with i.i.d. standard normal entries (Alg. 3,
step 2; the Hutchinson estimator of Sec. 3.3 needs mean 0 and variance 1).
It is realised here from a counter so that any block of it can be regenerated
on demand without storing it:

* Philox4x32-10, key = omega_seed (low word first);
* the call for data row ``i`` and sketch-row group ``g = r // 8`` uses the
  counter (i mod 2^32, i // 2^32, g, 0) and yields four 32-bit words w0..w3;
* word w_p gives one Box-Muller pair from two 16-bit uniforms:
  u1 = ((w_p & 0xFFFF) + 1) / 2^16 in (0, 1],  u2 = (w_p >> 16) / 2^16 in [0, 1),
  R = sqrt(-2 ln u1 / v),  z_{2p} = R cos(2 pi u2),  z_{2p+1} = R sin(2 pi u2);
* Omega[r, i] = z_{r mod 8}.

Box-Muller (Box and Muller, 1958) turns two uniforms into two independent
normals.  With 16-bit uniforms the plain transform (v = 1) has variance
``omega_variance()`` = ln N - ln(N!)/N = 1 - 9.87e-5 (N = 2^16), not 1; the
radius is therefore divided by sqrt(v) with v = omega_variance(), so that the
entries have mean 0 and variance exactly 1, as the Hutchinson estimator of
Sec. 3.3 assumes.  They are centred, symmetric and bounded by
sqrt(32 ln 2 / v) ~ 4.7098 (a sub-Gaussian test matrix, which is what
NA-Hutch++ requires).  The oracle evaluates the transform in binary64.
"""
from __future__ import annotations

import math

import numpy as np

from .philox import DOMAIN_OMEGA, philox4x32, seed_key

ROWS_PER_CALL = 8
UNIFORM_BITS = 16
_INV16 = 1.0 / 65536.0


def omega_variance():
    """Exact variance of one entry of the plain 16-bit Box-Muller transform
    (radius sqrt(-2 ln u1)): E[R^2] E[cos^2] with u1 uniform on the grid
    {1/N, ..., N/N}, N = 2^16, and E[cos^2(2 pi k / N)] = 1/2:
    Var = -(1/N) sum_{j=1..N} ln(j/N) = ln N - ln(N!)/N."""
    n = 1 << UNIFORM_BITS
    return math.log(n) - math.lgamma(n + 1) / n


def omega_bound():
    """Largest |Omega| entry: the radius at u1 = 1/N, sqrt(2 ln N / v)."""
    return math.sqrt(2.0 * UNIFORM_BITS * math.log(2.0) / omega_variance())


def _box_muller(words):
    """words: uint64 array (..., 4) of 32-bit words -> float64 (..., 8)."""
    lo = (words & np.uint64(0xFFFF)).astype(np.float64)
    hi = (words >> np.uint64(16)).astype(np.float64)
    u1 = (lo + 1.0) * _INV16
    u2 = hi * _INV16
    rad = np.sqrt(-2.0 * np.log(u1) / omega_variance())
    ang = 2.0 * np.pi * u2
    z = np.empty(words.shape[:-1] + (8,), dtype=np.float64)
    z[..., 0::2] = rad * np.cos(ang)
    z[..., 1::2] = rad * np.sin(ang)
    return z


def omega_block(omega_seed, ell, i0, count):
    """Omega[:, i0:i0+count] as an (ell x count) float64 array."""
    k0, k1 = seed_key(omega_seed)
    ngroups = (ell + ROWS_PER_CALL - 1) // ROWS_PER_CALL
    i = np.arange(i0, i0 + count, dtype=np.uint64)
    g = np.arange(ngroups, dtype=np.uint64)
    ii = i[None, :]
    gg = g[:, None]
    w0, w1, w2, w3 = philox4x32(ii & np.uint64(0xFFFFFFFF), ii >> np.uint64(32), gg, DOMAIN_OMEGA, k0, k1)
    words = np.stack([w0, w1, w2, w3], axis=-1)          # (ngroups, count, 4)
    z = _box_muller(words)                                # (ngroups, count, 8)
    z = np.transpose(z, (0, 2, 1)).reshape(ngroups * ROWS_PER_CALL, count)
    return np.ascontiguousarray(z[:ell])


def omega_entry_scalar(omega_seed, r, i):
    """One entry, from the scalar Philox and the math module (for brute-force
    cross-checks of ``omega_block``)."""
    from .philox import philox4x32_scalar
    key = seed_key(omega_seed)
    w = philox4x32_scalar((i & 0xFFFFFFFF, i >> 32, r // ROWS_PER_CALL, DOMAIN_OMEGA), key)
    p = (r % ROWS_PER_CALL) // 2
    u1 = ((w[p] & 0xFFFF) + 1) / 65536.0
    u2 = (w[p] >> 16) / 65536.0
    rad = math.sqrt(-2.0 * math.log(u1) / omega_variance())
    if r % 2 == 0:
        return rad * math.cos(2.0 * math.pi * u2)
    return rad * math.sin(2.0 * math.pi * u2)


def round_to_bf16(x):
    """Round-to-nearest-even of float32 values to bfloat16, returned as
    float64 (the operand rounding a bfloat16 contraction applies)."""
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    bits = (bits + np.uint64(0x7FFF) + ((bits >> np.uint64(16)) & np.uint64(1))) & np.uint64(0xFFFF0000)
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# FP8 (OCP e4m3) operands of the fp8 sketch form.
# e4m3: 1 sign, 4 exponent (bias 7), 3 mantissa bits; no infinities; largest
# finite magnitude 448 = 1.75 * 2^8; subnormals k * 2^-9, k = 1..7.
# --------------------------------------------------------------------------
E4M3_MAX = 448.0
OMEGA_FP8_EXP = -6     # Omega is stored as e4m3(Omega * 2^6) with scale 2^-6
MX_BLOCK = 32          # rows per shared scale of the data (microscaling block)


def round_to_e4m3(x):
    """Round-to-nearest-even onto the e4m3 grid, saturating at +-448
    (float64 in, float64 out)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    with np.errstate(divide="ignore"):
        _, E = np.frexp(a)                       # a = f * 2^E, f in [0.5, 1)
    e = np.maximum(E - 1, -6)                    # binade of a; subnormals share 2^-6's spacing
    step = np.ldexp(1.0, e - 3)
    q = np.round(a / step) * step                # numpy rounds half to even
    q = np.minimum(q, E4M3_MAX)
    return np.where(x < 0, -q, q)


def mx_block_exponent(amax):
    """Shared scale exponent of a block with largest magnitude amax:
    floor(log2 amax) - 7, so the scaled maximum lies in [128, 256) and no
    element saturates (with floor(log2 amax) - 8 the maximum could land in
    (448, 512) and lose up to 12.5%); clamped to the E8M0 range [-127, 127];
    -127 for an all-zero block."""
    amax = np.asarray(amax, dtype=np.float64)
    with np.errstate(divide="ignore"):
        _, E = np.frexp(amax)
    e = np.where(amax > 0, E - 1 - 7, -127)
    return np.clip(e, -127, 127)


def quantize_fp8_blocks(blk):
    """e4m3 data operand with one power-of-two scale per 32 consecutive rows of
    each column (rows counted from the first row of ``blk``, which the callers
    keep aligned to a multiple of 32); returns the dequantized float64 values."""
    blk = np.asarray(blk, dtype=np.float64)
    m, b = blk.shape
    out = np.empty_like(blk)
    for r0 in range(0, m, MX_BLOCK):
        part = blk[r0:r0 + MX_BLOCK]
        e = mx_block_exponent(np.max(np.abs(part), axis=0))
        sc = np.ldexp(1.0, e)
        out[r0:r0 + MX_BLOCK] = round_to_e4m3(part / sc) * sc
    return out


def quantize_fp8_omega(om):
    """e4m3 test-matrix operand: e4m3(Omega * 2^6) * 2^-6."""
    sc = math.ldexp(1.0, OMEGA_FP8_EXP)
    return round_to_e4m3(np.asarray(om, dtype=np.float64) / sc) * sc

