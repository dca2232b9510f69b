"""Seeded synthetic colour images and impulsive-noise models.

The paper's test images are not available, so every workload here is
synthetic: a smooth random colour field with straight edges, corrupted by one
of three impulsive-noise models.  This module holds no part of the filter's
arithmetic; the GPU path and the CPU oracle both take their inputs from it.

Image recipe ``smooth_image(M, N, rng)``:
  1. per channel, the sum of 8 plane waves ``a sin(2 pi f (c cos phi + r sin phi) + psi)``
     with a ~ U(0.5, 1), f ~ U(1/128, 1/16) cycles/pixel, phi ~ U(0, pi),
     psi ~ U(0, 2 pi), min-max scaled to [0, 255];
  2. 20 straight edges: a line through (U(0, N), U(0, M)) at angle U(0, pi),
     with a colour offset U(-60, 60)^3 added on one side;
  3. clipped to [0, 255] and rounded to uint8.

Noise models (masks are drawn first, then the replacement values):
  * ``noise_uncorrelated(x, phi)``: each channel independently replaced with
    probability phi by a value uniform in {0..255};
  * ``noise_correlated(x, phi)``: each pixel replaced with probability phi by a
    colour uniform in {0..255}^3;
  * ``noise_eq8(x, phi)``: the correlated impulsive model of eq. (8), with
    channel probabilities phi_1 = phi_2 = phi_3 = 0.25 (Section III): a pixel
    is corrupted with probability phi, then R only, G only, B only or all three
    channels with probability 1/4 each.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng_for", "smooth_image", "noise_uncorrelated", "noise_correlated", "noise_eq8",
    "dither_float", "image_uncorr", "image_corr", "float_batch", "mixed_batch_specs",
    "mixed_batch_images",
]

# Row chunk for the large-frame generator (bounds the float32 temporaries).
_CHUNK_ROWS = 512


def rng_for(*key: int) -> np.random.Generator:
    """PCG64 generator seeded from an integer key (the first element is 1009)."""
    return np.random.default_rng([1009, *[int(k) for k in key]])


def smooth_image(M: int, N: int, rng: np.random.Generator) -> np.ndarray:
    """Seeded smooth colour field with 20 straight edges, uint8 (M, N, 3)."""
    waves = []
    for _ in range(3):
        a = rng.uniform(0.5, 1.0, 8)
        f = rng.uniform(1.0 / 128, 1.0 / 16, 8)
        phi = rng.uniform(0.0, np.pi, 8)
        psi = rng.uniform(0.0, 2 * np.pi, 8)
        waves.append((a, f, phi, psi))
    edges = []
    for _ in range(20):
        c0 = rng.uniform(0, N)
        r0 = rng.uniform(0, M)
        ang = rng.uniform(0, np.pi)
        off = rng.uniform(-60, 60, 3)
        edges.append((c0, r0, ang, off))

    cols = np.arange(N, dtype=np.float64)
    field = np.empty((M, N, 3), np.float32)
    for ch, (a, f, phi, psi) in enumerate(waves):
        # sin(u + v) = sin u cos v + cos u sin v, with u along columns and v along rows
        ucol = 2 * np.pi * f[:, None] * np.cos(phi)[:, None] * cols[None, :]  # (8, N)
        su, cu = np.sin(ucol).astype(np.float32), np.cos(ucol).astype(np.float32)
        for r0 in range(0, M, _CHUNK_ROWS):
            rows = np.arange(r0, min(M, r0 + _CHUNK_ROWS), dtype=np.float64)
            vrow = 2 * np.pi * f[:, None] * np.sin(phi)[:, None] * rows[None, :] + psi[:, None]
            sv = (a[:, None] * np.sin(vrow)).astype(np.float32)  # (8, R)
            cv = (a[:, None] * np.cos(vrow)).astype(np.float32)
            field[r0:r0 + rows.shape[0], :, ch] = sv.T @ cu + cv.T @ su
    lo = field.reshape(-1, 3).min(axis=0)
    hi = field.reshape(-1, 3).max(axis=0)
    scale = (255.0 / np.maximum(hi - lo, 1e-6)).astype(np.float32)
    out = np.empty((M, N, 3), np.uint8)
    ec0 = np.array([e[0] for e in edges], np.float32)
    er0 = np.array([e[1] for e in edges], np.float32)
    esin = np.array([np.sin(e[2]) for e in edges], np.float32)
    ecos = np.array([np.cos(e[2]) for e in edges], np.float32)
    eoff = np.array([e[3] for e in edges], np.float32)  # (20, 3)
    colterm = (cols.astype(np.float32)[:, None] - ec0[None, :]) * esin[None, :]  # (N, 20)
    for r0 in range(0, M, _CHUNK_ROWS // 4):
        r1 = min(M, r0 + _CHUNK_ROWS // 4)
        blk = (field[r0:r1] - lo) * scale
        rowterm = (np.arange(r0, r1, dtype=np.float32)[:, None] - er0[None, :]) * ecos[None, :]
        side = (colterm[None, :, :] - rowterm[:, None, :] > 0).astype(np.float32)  # (R, N, 20)
        blk += side @ eoff
        np.clip(blk, 0, 255, out=blk)
        out[r0:r1] = np.rint(blk).astype(np.uint8)
    return out


def noise_uncorrelated(x: np.ndarray, phi: float, rng: np.random.Generator) -> np.ndarray:
    """Each channel independently replaced with probability phi by U{0..255}."""
    mask = rng.random(x.shape) < phi
    vals = rng.integers(0, 256, x.shape, dtype=np.uint8)
    return np.where(mask, vals, x).astype(np.uint8)


def noise_correlated(x: np.ndarray, phi: float, rng: np.random.Generator) -> np.ndarray:
    """Each pixel replaced with probability phi by a colour uniform in {0..255}^3."""
    mask = rng.random(x.shape[:-1]) < phi
    vals = rng.integers(0, 256, x.shape, dtype=np.uint8)
    return np.where(mask[..., None], vals, x).astype(np.uint8)


def noise_eq8(x: np.ndarray, phi: float, rng: np.random.Generator,
              channel_probs=(0.25, 0.25, 0.25)) -> np.ndarray:
    """Impulsive noise of eq. (8): R, G, B alone or all three, after a per-pixel draw."""
    hit = rng.random(x.shape[:-1]) < phi
    cum = np.cumsum([channel_probs[0], channel_probs[1], channel_probs[2]])
    which = np.searchsorted(cum, rng.random(x.shape[:-1]), side="right")  # 0, 1, 2 or 3 (all)
    vals = rng.integers(0, 256, x.shape, dtype=np.uint8)
    chan = np.arange(3)
    replace = hit[..., None] & ((which[..., None] == chan) | (which[..., None] == 3))
    return np.where(replace, vals, x).astype(np.uint8)


def dither_float(x_u8: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """uint8 image -> float32 in [0, 1] with U(-0.5, 0.5)/255 dither."""
    y = x_u8.astype(np.float64) / 255.0 + rng.uniform(-0.5, 0.5, x_u8.shape) / 255.0
    return np.clip(y, 0.0, 1.0).astype(np.float32)


# ---------------------------------------------------------------- workloads

def image_uncorr(M: int, N: int, phi: float, key: int = 0) -> np.ndarray:
    """One smooth image with uncorrelated per-channel impulsive noise."""
    rng = rng_for(1, key, M, N)
    return noise_uncorrelated(smooth_image(M, N, rng), phi, rng)


def image_corr(M: int, N: int, phi: float, key: int = 0) -> np.ndarray:
    """One smooth image with per-pixel correlated impulsive noise."""
    rng = rng_for(2, key, M, N)
    return noise_correlated(smooth_image(M, N, rng), phi, rng)


def float_batch(B: int, M: int, N: int, phi: float, key: int = 0) -> np.ndarray:
    """B float32 images in [0, 1]: smooth image, correlated noise, dither."""
    out = np.empty((B, M, N, 3), np.float32)
    for b in range(B):
        rng = rng_for(4, key, b)
        out[b] = dither_float(noise_correlated(smooth_image(M, N, rng), phi, rng), rng)
    return out


def mixed_batch_specs(count: int = 256, key: int = 0, max_M: int = 1536, max_N: int = 2048):
    """Specs of a mixed batch: sizes uniform in 64..max, window 3 or 5, BVDF or
    DDF(p = 0.25), eq. (8) noise rate uniform in [0.05, 0.30]."""
    rng = rng_for(3, key)
    specs = []
    for i in range(count):
        N = int(rng.integers(64, max_N + 1))
        M = int(rng.integers(64, max_M + 1))
        w = int(rng.choice([3, 5]))
        kind = int(rng.integers(0, 2))
        phi = float(rng.uniform(0.05, 0.30))
        specs.append(dict(index=i, M=M, N=N, window=w, kind=kind, p=0.25, phi=phi))
    return specs


def mixed_batch_images(specs, key: int = 0, workers: int = 8):
    """The uint8 images of ``mixed_batch_specs`` (generated in a thread pool;
    each image has its own seeded generator, so the result does not depend on
    the number of workers)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(s):
        rng = rng_for(3, key, 1000 + s["index"])
        return noise_eq8(smooth_image(s["M"], s["N"], rng), s["phi"], rng)

    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        return list(ex.map(one, specs))
