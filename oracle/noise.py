"""CPU oracle of the correlated impulsive noise model of eq. (8) (Section III)
and of the MAE / PSNR measures.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check
and the benchmark's CPU-baseline leg may import this module; it shares no code
with the GPU library.

Random numbers: Philox4x32-10, written here from its published definition
(Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC 2011): ten rounds of two 32 x 32 -> 64-bit multiplications by 0xD2511F53 and
0xCD9E8D57 on counter words 0 and 2, with the key bumped by the Weyl constants
0x9E3779B9 and 0xBB67AE85 between rounds.  Pixel i (flat index over
B x M x N) uses counter (i mod 2^32, i div 2^32, 0, 0) and key
(seed mod 2^32, seed div 2^32).
"""
from __future__ import annotations

import math

import numpy as np

_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(counter, key):
    """Philox4x32-10 of counters (n, 4) uint32 under key (2,) uint32 -> (n, 4) uint32."""
    c = [np.asarray(counter, np.uint64)[:, j].copy() for j in range(4)]
    k0, k1 = np.uint64(int(key[0]) & 0xFFFFFFFF), np.uint64(int(key[1]) & 0xFFFFFFFF)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(_W0)) & _MASK
            k1 = (k1 + np.uint64(_W1)) & _MASK
        p0 = np.uint64(_M0) * c[0]  # < 2^64: exact in uint64
        p1 = np.uint64(_M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=1).astype(np.uint32)


def _threshold(p):
    """floor(p 2^32) for p in [0, 1] (p 2^32 is an exact binary64 scaling)."""
    return min(int(math.floor(p * 4294967296.0)), 1 << 32)


def pixel_draws(npix, seed):
    """The Philox block of every pixel 0 .. npix-1, (npix, 4) uint32."""
    i = np.arange(npix, dtype=np.uint64)
    ctr = np.stack([i & _MASK, i >> np.uint64(32), np.zeros_like(i), np.zeros_like(i)], axis=1)
    return philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))


def noise_eq8(clean, phi, phi_rgb=(0.25, 0.25, 0.25), seed=0):
    """eq. (8): with probability phi a pixel is corrupted; then red only, green
    only, blue only (probabilities phi_rgb) or all three channels (the rest)
    take the values of r, uniform in {0..255}^3."""
    x = np.asarray(clean, np.uint8)
    flat = x.reshape(-1, 3).copy()
    u = pixel_draws(flat.shape[0], int(seed)).astype(np.uint64)
    hit = u[:, 0] < np.uint64(_threshold(phi))
    t1 = _threshold(phi_rgb[0])
    t2 = _threshold(phi_rgb[0] + phi_rgb[1])
    t3 = _threshold(phi_rgb[0] + phi_rgb[1] + phi_rgb[2])
    pat = np.where(u[:, 1] < np.uint64(t1), 0, np.where(u[:, 1] < np.uint64(t2), 1,
                                                     np.where(u[:, 1] < np.uint64(t3), 2, 3)))
    for k in range(3):
        r = ((u[:, 2] >> np.uint64(8 * k)) & np.uint64(0xFF)).astype(np.uint8)
        sel = hit & ((pat == k) | (pat == 3))
        flat[sel, k] = r[sel]
    return flat.reshape(x.shape)


def quality(y, ref):
    """Per image: MAE = sum |y - ref| / 3MN and PSNR = 10 log10(255^2 / MSE),
    MSE = sum (y - ref)^2 / 3MN (inf for identical images).  Returns two
    float64 arrays of length B (images (B, M, N, 3) or one (M, N, 3))."""
    a = np.asarray(y, np.int64)
    b = np.asarray(ref, np.int64)
    if a.ndim == 3:
        a, b = a[None], b[None]
    d = (a - b).reshape(a.shape[0], -1)
    n = float(d.shape[1])
    s1 = np.abs(d).sum(axis=1)
    s2 = (d * d).sum(axis=1)
    mae = np.array([float(v) / n for v in s1])
    psnr = np.array([math.inf if v == 0 else 10.0 * math.log10(255.0 * 255.0 * n / float(v))
                     for v in s2])
    return mae, psnr
