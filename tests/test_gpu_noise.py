"""GPU eq. (8) noise and MAE / PSNR against the CPU oracle: the noise is
bit-exact (both sides implement Philox4x32-10 from its definition), MAE is
exact (integer sums), PSNR within 1e-12 relative (device vs host log10)."""
import math

import numpy as np
import pytest

from oracle import noise as onoise
from paper_1009_0958_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1009_0958_amd import odf  # noqa: E402

DEV = "cuda:0"


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 7, 5), (2, 33, 65), (3, 64, 64), (1, 300, 517)])
@pytest.mark.parametrize("phi,rgb,seed", [(0.0, (0.25, 0.25, 0.25), 1), (0.1, (0.25, 0.25, 0.25), 2),
                                          (0.15, (0.25, 0.25, 0.25), 3), (1.0, (0.5, 0.2, 0.1), 4),
                                          (0.3, (0.0, 0.0, 0.0), (5 << 32) | 9)])
def test_noise_bit_exact(shape, phi, rgb, seed):
    print("case: shape=%s phi=%s rgb=%s seed=%d" % (shape, phi, rgb, seed), flush=True)
    clean = np.random.default_rng(7).integers(0, 256, shape + (3,)).astype(np.uint8)
    got = odf.noise_eq8(_gpu(clean), phi, rgb, seed).cpu().numpy()
    assert np.array_equal(got, onoise.noise_eq8(clean, phi, rgb, seed))


def test_noise_in_place_and_full_frame():
    clean = synth.smooth_image(1024, 1024, synth.rng_for(8, 0))
    x = _gpu(clean[None])
    odf.noise_eq8(x, 0.15, seed=77, out=x)
    assert np.array_equal(x.cpu().numpy()[0], onoise.noise_eq8(clean, 0.15, seed=77))


def test_noise_unaligned_views():
    """Buffers off 4-byte alignment take the pixel-by-pixel form (aligned ones
    four pixels per thread); the noise is the same."""
    clean = np.random.default_rng(9).integers(0, 256, (1, 37, 41, 3)).astype(np.uint8)
    ref = onoise.noise_eq8(clean, 0.2, seed=11)
    buf = torch.zeros(clean.size + 1, dtype=torch.uint8, device=DEV)
    x = buf[1:].view(clean.shape)
    x.copy_(_gpu(clean))
    assert np.array_equal(odf.noise_eq8(x, 0.2, seed=11).cpu().numpy(), ref)
    obuf = torch.zeros(clean.size + 2, dtype=torch.uint8, device=DEV)
    out = obuf[2:].view(clean.shape)
    odf.noise_eq8(_gpu(clean), 0.2, seed=11, out=out)
    assert np.array_equal(out.cpu().numpy(), ref)
    assert np.array_equal(odf.noise_eq8(_gpu(clean), 0.2, seed=11).cpu().numpy(), ref)


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 5, 7), (1, 64, 64), (4, 33, 48), (1, 1024, 1024)])
def test_quality_matches_oracle(shape):
    print("case: quality shape=%s" % (shape,), flush=True)
    rng = np.random.default_rng(shape[1])
    ref = rng.integers(0, 256, shape + (3,)).astype(np.uint8)
    y = ref.copy()
    mask = rng.random(y.shape) < 0.2
    y[mask] = rng.integers(0, 256, mask.sum())
    mae, psnr = (t.cpu().numpy() for t in odf.quality(_gpu(y), _gpu(ref)))
    omae, opsnr = onoise.quality(y, ref)
    assert np.array_equal(mae, omae)
    for a, b in zip(psnr, opsnr):
        assert (math.isinf(a) and math.isinf(b)) or a == pytest.approx(b, rel=1e-12)


def test_quality_unaligned_and_identical():
    ref = np.random.default_rng(3).integers(0, 256, (2, 16, 16, 3)).astype(np.uint8)
    y = ref.copy()
    y[1, 3, 4, 2] ^= 0x55
    buf_y = torch.empty(y.size + 1, dtype=torch.uint8, device=DEV)
    buf_r = torch.empty(ref.size + 1, dtype=torch.uint8, device=DEV)
    buf_y[1:] = _gpu(y.ravel())
    buf_r[1:] = _gpu(ref.ravel())
    yv, rv = buf_y[1:].view(y.shape), buf_r[1:].view(ref.shape)  # 1-byte offset: byte path
    mae, psnr = (t.cpu().numpy() for t in odf.quality(yv, rv))
    omae, opsnr = onoise.quality(y, ref)
    assert np.array_equal(mae, omae) and mae[0] == 0 and math.isinf(psnr[0])
    assert psnr[1] == pytest.approx(opsnr[1], rel=1e-12)


def test_noise_keeps_the_input_shape():
    clean = np.random.default_rng(9).integers(0, 256, (20, 30, 3)).astype(np.uint8)
    got = odf.noise_eq8(_gpu(clean), 0.2, seed=3)
    assert tuple(got.shape) == (20, 30, 3)
    assert np.array_equal(got.cpu().numpy(), onoise.noise_eq8(clean, 0.2, seed=3))
