"""The Gaussian test matrix Omega of the oracle (test infrastructure only).

The paper draws Omega (l x m) with i.i.d. standard normal entries (Alg. 3,
step 2); the Hutchinson estimator of Sec. 3.3 needs mean 0 and variance 1,
and a sub-Gaussian distribution suffices for NA-Hutch++.  It is realised here
from a counter so that any block can be regenerated on demand without being
stored, and from a table of quantiles so that every reduced-precision form
holds exactly the rounding of the same binary64 value:

* Philox4x32-10, key = omega_seed (low word first);
* the call for data row ``i`` and sketch-row group ``g = r // 8`` uses the
  counter (i mod 2^32, i // 2^32, g, 0) and yields four 32-bit words w0..w3,
  i.e. eight 16-bit halves h_{2p} = w_p & 0xFFFF, h_{2p+1} = w_p >> 16;
* Omega[r, i] = (-1)^s T[k] for h = h_{r mod 8}, s = h >> 15 (bit 15) and
  k = (h >> 5) & 1023 (bits 14..5; bits 4..0 are not used);
* T[k] = c Phi^{-1}((1 + (k + 1/2) / 1024) / 2), k = 0..1023, the quantile of
  |N(0, 1)| at the middle of the k-th of 1024 equiprobable bins, with c the
  constant that makes the mean of T^2 exactly 1.

So each entry takes one of 2048 equiprobable values, symmetric about 0: the
standard normal distribution quantised to 2048 atoms (it is within 1/2048 of
the normal CDF everywhere), with mean 0 and variance exactly 1 and bounded by
T[1023] ~ 3.49 (a sub-Gaussian test matrix).  The quantiles are the binary64
values of ``scipy.special.ndtri``.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ndtri

from .philox import DOMAIN_OMEGA, philox4x32, seed_key

ROWS_PER_CALL = 8
TABLE_BITS = 10
TABLE_SIZE = 1 << TABLE_BITS
INDEX_SHIFT = 5


def _half_normal_quantiles():
    p = 0.5 * (1.0 + (np.arange(TABLE_SIZE, dtype=np.float64) + 0.5) / TABLE_SIZE)
    return ndtri(p)


def omega_scale():
    """c = 1 / sqrt(mean_k Q_k^2) for the unscaled quantiles Q_k."""
    q = _half_normal_quantiles()
    return 1.0 / math.sqrt(float(np.mean(q * q)))


_TABLE = _half_normal_quantiles() * omega_scale()


def omega_table():
    """The 1024 magnitudes T[k] (binary64, increasing)."""
    return _TABLE.copy()


def omega_bound():
    """Largest |Omega| entry: T[1023]."""
    return float(_TABLE[-1])


def omega_from_halves(h):
    """Entries for 16-bit halves h (integer array): (-1)^(h >> 15) T[(h >> 5) & 1023]."""
    h = np.asarray(h, dtype=np.uint64)
    k = ((h >> np.uint64(INDEX_SHIFT)) & np.uint64(TABLE_SIZE - 1)).astype(np.int64)
    z = _TABLE[k]
    return np.where((h >> np.uint64(15)) & np.uint64(1), -z, z)


def _halves(words):
    """words: uint64 array (..., 4) of 32-bit words -> (..., 8) 16-bit halves."""
    h = np.empty(words.shape[:-1] + (8,), dtype=np.uint64)
    h[..., 0::2] = words & np.uint64(0xFFFF)
    h[..., 1::2] = words >> np.uint64(16)
    return h


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
    z = omega_from_halves(_halves(words))                 # (ngroups, count, 8)
    z = np.transpose(z, (0, 2, 1)).reshape(ngroups * ROWS_PER_CALL, count)
    return np.ascontiguousarray(z[:ell])


def omega_entry_scalar(omega_seed, r, i):
    """One entry, from the scalar Philox and a direct quantile evaluation (for
    brute-force cross-checks of ``omega_block``)."""
    from .philox import philox4x32_scalar
    key = seed_key(omega_seed)
    w = philox4x32_scalar((i & 0xFFFFFFFF, i >> 32, r // ROWS_PER_CALL, DOMAIN_OMEGA), key)
    q = r % ROWS_PER_CALL
    h = (w[q // 2] >> (16 * (q % 2))) & 0xFFFF
    k = (h >> INDEX_SHIFT) & (TABLE_SIZE - 1)
    z = omega_scale() * float(ndtri(0.5 * (1.0 + (k + 0.5) / TABLE_SIZE)))
    return -z if h >> 15 else z


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

