"""Pins of the noise and quality oracle (eq. 8 and the MAE / PSNR measures of
Section III): published known-answer vectors of the generator, the
probabilities of eq. (8) and closed-form MAE / PSNR values."""
import math

import numpy as np
import pytest

from oracle import noise


def test_philox_known_answers():
    """Known-answer vectors published with Philox4x32-10 (Random123)."""
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, out in cases:
        got = noise.philox4x32_10(np.array([ctr], np.uint32), key)[0]
        assert tuple(int(v) for v in got) == out


def test_pixel_draws_use_flat_index_and_seed():
    d = noise.pixel_draws(3, (7 << 32) | 5)
    ref = noise.philox4x32_10(np.array([[2, 0, 0, 0]], np.uint32), (5, 7))[0]
    assert np.array_equal(d[2], ref)


@pytest.mark.parametrize("phi", [0.10, 0.15, 0.5])
def test_eq8_probabilities(phi):
    """Corrupted fraction phi; given corruption, red / green / blue only with
    0.25 each and all three with 0.25; replaced values uniform on {0..255}."""
    n = 400000
    clean = np.zeros((1, 400, 1000, 3), np.uint8)
    clean[:] = (1, 2, 3)  # a colour no draw... except r itself; count by pattern below
    u = noise.pixel_draws(n, 99).astype(np.uint64)
    x = noise.noise_eq8(clean, phi, seed=99).reshape(-1, 3)
    hit = u[:, 0] < np.uint64(math.floor(phi * 2 ** 32))
    frac = hit.mean()
    assert abs(frac - phi) < 5 * math.sqrt(phi * (1 - phi) / n)
    pat = np.minimum(u[hit, 1] // np.uint64(1 << 30), 3)
    for k in range(4):
        f = (pat == k).mean()
        assert abs(f - 0.25) < 5 * math.sqrt(0.25 * 0.75 / hit.sum())
    # unhit pixels are copies; hit pixels differ from the clean colour only in
    # the channels their pattern selects
    assert np.array_equal(x[~hit], np.broadcast_to(clean.reshape(-1, 3)[0], x[~hit].shape))
    sel = x[hit] != clean.reshape(-1, 3)[0]
    for k in range(3):
        changed = sel[:, k]
        allowed = (pat == k) | (pat == 3)
        assert not np.any(changed & ~allowed)
    r = x[hit][pat == 3].astype(np.int64).ravel()
    hist = np.bincount(r, minlength=256)
    exp = r.size / 256
    chi2 = ((hist - exp) ** 2 / exp).sum()
    assert chi2 < 255 + 6 * math.sqrt(2 * 255)


def test_eq8_edge_cases():
    rng = np.random.default_rng(3)
    clean = rng.integers(0, 256, (2, 9, 11, 3)).astype(np.uint8)
    assert np.array_equal(noise.noise_eq8(clean, 0.0, seed=1), clean)
    red = noise.noise_eq8(clean, 1.0, (1.0, 0.0, 0.0), seed=1)
    assert np.array_equal(red[..., 1:], clean[..., 1:])
    u = noise.pixel_draws(clean.size // 3, 1)
    assert np.array_equal(red[..., 0].ravel(), (u[:, 2] & 0xFF).astype(np.uint8))
    allc = noise.noise_eq8(clean, 1.0, (0.0, 0.0, 0.0), seed=1).reshape(-1, 3)
    for k in range(3):
        assert np.array_equal(allc[:, k], ((u[:, 2] >> (8 * k)) & 0xFF).astype(np.uint8))
    assert not np.array_equal(noise.noise_eq8(clean, 0.5, seed=2), noise.noise_eq8(clean, 0.5, seed=3))


def test_quality_closed_forms():
    a = np.full((2, 4, 5, 3), 100, np.uint8)
    mae, psnr = noise.quality(a, a)
    assert (mae == 0).all() and np.isinf(psnr).all()
    b = a.copy()
    b[0] += 1
    b[1, 0, 0, 0] = 110  # one value off by 10 of 60
    mae, psnr = noise.quality(b, a)
    assert mae[0] == 1.0 and psnr[0] == pytest.approx(20 * math.log10(255.0), rel=1e-15)
    assert mae[1] == pytest.approx(10 / 60, rel=1e-15)
    assert psnr[1] == pytest.approx(10 * math.log10(255.0 ** 2 * 60 / 100), rel=1e-15)


def test_expected_error_of_eq8_on_grey():
    """A mid-grey image o = 128: the expected share of replaced channel values
    is phi (0.75 * 1 + 0.25 * 3) / 3 = phi / 2, and a uniform r has
    E|r - 128| = 64 and E(r - 128)^2 = (sum_{k=-128}^{127} k^2) / 256."""
    phi = 0.2
    clean = np.full((1, 1000, 1000, 3), 128, np.uint8)
    mae, psnr = noise.quality(noise.noise_eq8(clean, phi, seed=11), clean)
    e_abs = 64.0
    e_sq = sum(k * k for k in range(-128, 128)) / 256.0
    # relative standard deviations at 10^6 pixels: ~0.3 % (MAE), ~0.35 % (MSE);
    # the bounds are ~6 of them
    assert mae[0] == pytest.approx(phi / 2 * e_abs, rel=0.02)
    mse = 255.0 ** 2 / 10 ** (psnr[0] / 10)
    assert mse == pytest.approx(phi / 2 * e_sq, rel=0.02)
