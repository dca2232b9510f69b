"""Seeded synthetic inputs: determinism, ranges and noise rates."""
import numpy as np

from paper_1009_0958_amd import synth


def test_smooth_image_deterministic_and_full_range():
    a = synth.smooth_image(96, 128, synth.rng_for(0))
    b = synth.smooth_image(96, 128, synth.rng_for(0))
    c = synth.smooth_image(96, 128, synth.rng_for(1))
    assert a.dtype == np.uint8 and a.shape == (96, 128, 3)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() <= 5 and a.max() >= 250


def test_noise_rates():
    x = np.full((400, 500, 3), 128, np.uint8)
    rng = np.random.default_rng(0)
    u = synth.noise_uncorrelated(x, 0.1, rng)
    assert abs((u != 128).mean() - 0.1 * 255 / 256) < 0.005
    c = synth.noise_correlated(x, 0.2, rng)
    hit = (c != 128).any(-1)
    assert abs(hit.mean() - 0.2) < 0.005
    e = synth.noise_eq8(x, 0.3, rng)
    per_pixel = (e != 128).sum(-1)
    # single-channel hits are 3/4 of corrupted pixels, all-channel hits 1/4
    assert abs((per_pixel == 1).mean() - 0.3 * 0.75) < 0.01
    assert abs((per_pixel == 3).mean() - 0.3 * 0.25 * (255 / 256) ** 3) < 0.01


def test_float_batch_range():
    f = synth.float_batch(2, 32, 40, 0.1)
    assert f.dtype == np.float32 and f.shape == (2, 32, 40, 3)
    assert f.min() >= 0.0 and f.max() <= 1.0


def test_mixed_batch_specs():
    s = synth.mixed_batch_specs(256)
    assert len(s) == 256
    assert all(64 <= d["M"] <= 1536 and 64 <= d["N"] <= 2048 for d in s)
    assert {d["window"] for d in s} == {3, 5} and {d["kind"] for d in s} == {0, 1}
    assert all(0.05 <= d["phi"] <= 0.30 for d in s)
