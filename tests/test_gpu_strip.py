"""The strip form of the forward filter (configs 4 and 5: strips of 8 and of 3
bands): bitwise equal to the tile form, and against the FP64 oracle directly."""
import numpy as np
import pytest

import oracle
from paper_1009_0958_amd import synth
from parity import check_selection, source_pixels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1009_0958_amd import odf  # noqa: E402

DEV = "cuda:0"
BVDF, DDF = odf.BVDF, odf.DDF
EXACT, MINIMAX, RGB = odf.EXACT, odf.MINIMAX, odf.RGB
STRIP = 4
STRIPS = [odf.STRIP, odf.SHORT_STRIP]


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _run(x, window, kind, p, dist, cfg):
    u8 = x.dtype == torch.uint8
    saved = odf.tune_get(window, kind, dist, u8)
    odf.tune_set(window, kind, dist, u8, cfg)
    try:
        out, idx = odf.filter(x, window, kind, p, dist)
        torch.cuda.synchronize()
    finally:
        odf.tune_set(window, kind, dist, u8, saved)
    return out.cpu().numpy(), idx.cpu().numpy()


def _image(shape, u8, key):
    B, M, N = shape
    img = np.stack([synth.image_corr(M, N, 0.15, key=key + b) for b in range(B)])
    if u8:
        return img
    return (img.astype(np.float32) / 255.0).astype(np.float32)


# shapes: one strip, several strips down and across (124 output rows per
# strip), ragged on both axes, a batch of images, and the degenerate ones
SHAPES = [(1, 1, 1), (1, 1, 97), (1, 130, 1), (1, 5, 7), (1, 124, 28), (1, 125, 29),
          (1, 300, 190), (2, 257, 61), (1, 40, 700)]


@pytest.mark.parametrize("cfg", STRIPS)
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("window,kind,p", [(3, BVDF, 0.0), (3, DDF, 0.25), (5, BVDF, 0.0),
                                           (5, DDF, 0.25), (5, DDF, 0.5), (7, BVDF, 0.0),
                                           (7, DDF, 0.25), (9, BVDF, 0.0)])
def test_strip_equals_tile_u8(shape, window, kind, p, cfg):
    img = _image(shape, True, 7)
    x = _gpu(img)
    for dist in (EXACT, MINIMAX, RGB):
        print("case: strip %d u8 shape=%s w=%d kind=%d p=%s dist=%d"
              % (cfg, shape, window, kind, p, dist), flush=True)
        o_t, i_t = _run(x, window, kind, p, dist, 2)
        o_s, i_s = _run(x, window, kind, p, dist, cfg)
        assert np.array_equal(i_s, i_t)
        assert np.array_equal(o_s, o_t)


@pytest.mark.parametrize("cfg", STRIPS)
@pytest.mark.parametrize("shape", [(1, 130, 61), (2, 257, 45), (1, 3, 3)])
@pytest.mark.parametrize("window,kind,p", [(3, DDF, 0.5), (5, BVDF, 0.0), (5, DDF, 0.25),
                                           (7, BVDF, 0.0), (7, DDF, 0.5)])
def test_strip_equals_tile_f32(shape, window, kind, p, cfg):
    img = _image(shape, False, 11)
    x = _gpu(img)
    for dist in (EXACT, MINIMAX, RGB):
        print("case: strip %d f32 shape=%s w=%d kind=%d p=%s dist=%d"
              % (cfg, shape, window, kind, p, dist), flush=True)
        o_t, i_t = _run(x, window, kind, p, dist, 2)
        o_s, i_s = _run(x, window, kind, p, dist, cfg)
        assert np.array_equal(i_s, i_t)
        assert np.array_equal(o_s, o_t)


@pytest.mark.parametrize("window,kind,p,dist", [(5, DDF, 0.25, EXACT), (5, BVDF, 0.0, MINIMAX),
                                                (3, DDF, 0.5, RGB), (7, DDF, 0.25, EXACT),
                                                (9, BVDF, 0.0, EXACT)])
def test_strip_oracle(window, kind, p, dist):
    """The strip forms against the oracle on an image of three long strips down."""
    img = synth.image_corr(290, 75, 0.2, key=3)
    _, _, _, _, oO = oracle.filter(img, window, kind, p, dist, 4, aggregates=True)
    for cfg in STRIPS:
        print("case: strip %d oracle w=%d kind=%d p=%s dist=%d" % (cfg, window, kind, p, dist),
              flush=True)
        out, idx = _run(_gpu(img), window, kind, p, dist, cfg)
        n_mis, n = check_selection(idx, oO)
        print("mismatch %d / %d" % (n_mis, n))
        assert np.array_equal(out.reshape(-1, 3), source_pixels(img, idx, window).reshape(-1, 3))


def test_strip_not_offered():
    """The strip form covers BVDF and DDF at 3x3 to 7x7, BVDF at 9x9 on uint8 and
    the centre-weighted kinds at 3x3 to 7x7."""
    for window, kind, u8 in [(9, DDF, True), (9, BVDF, False)]:
        for cfg in STRIPS:
            with pytest.raises(odf.ODFError):
                odf.tune_set(window, kind, EXACT, u8, cfg)


def _run_cw(x, window, kind, dist, cfg, level):
    """ACWDDF (lambda = 2, T = 10.8) or a centre-weighted filter at `level` on config cfg."""
    u8 = x.dtype == torch.uint8
    saved = odf.tune_get(window, kind, dist, u8)
    odf.tune_set(window, kind, dist, u8, cfg)
    try:
        if kind == odf.ACWDDF:
            out, idx = odf.acwddf(x, window, dist, 4, 2, 10.8)
        else:
            out, idx = odf.cw_filter(x, window, kind, level, dist)
        torch.cuda.synchronize()
    finally:
        odf.tune_set(window, kind, dist, u8, saved)
    return out.cpu().numpy(), idx.cpu().numpy()


@pytest.mark.parametrize("cfg", STRIPS)
@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 5, 7), (1, 130, 61), (2, 257, 45), (1, 40, 300)])
@pytest.mark.parametrize("window", [3, 5, 7])
@pytest.mark.parametrize("u8", [True, False])
def test_strip_equals_tile_centre_weighted(shape, window, u8, cfg):
    """ACWDDF (its four keys per window and the switching statistic) and the
    centre-weighted filters CWDDF^k and CWVMF^k on the strip form, bitwise equal
    to their 32 x 16 tiles."""
    img = _image(shape, u8, 13)
    x = _gpu(img)
    for kind, dists, level in [(odf.ACWDDF, (EXACT, MINIMAX, RGB), 0), (odf.CWDDF, (EXACT, RGB), 2),
                               (odf.CWVMF, (RGB,), window)]:
        for dist in dists:
            print("case: strip %d cw u8=%s shape=%s w=%d kind=%d dist=%d level=%d"
                  % (cfg, u8, shape, window, kind, dist, level), flush=True)
            o_t, i_t = _run_cw(x, window, kind, dist, 2, level)
            o_s, i_s = _run_cw(x, window, kind, dist, cfg, level)
            assert np.array_equal(i_s, i_t)
            assert np.array_equal(o_s, o_t)
