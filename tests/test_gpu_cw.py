"""GPU parity of the centre-weighted filters (Section III, eq. 9: CWVMF^k and
CWDDF^k at one smoothing level), through the C ABI, against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1009_0958_amd import synth
from parity import check_selection, source_pixels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1009_0958_amd import odf  # noqa: E402

DEV = "cuda:0"
EXACT, MINIMAX, RGB = odf.EXACT, odf.MINIMAX, odf.RGB


def _run(img, window, kind, level, dist, q=4):
    print("case: %s w=%d kind=%d level=%d dist=%d" % (img.shape, window, kind, level, dist),
          flush=True)
    x = torch.from_numpy(np.ascontiguousarray(img)).to(DEV)
    out, idx = odf.cw_filter(x, window, kind, level, dist, q)
    out, idx = out.cpu().numpy(), idx.cpu().numpy()
    _, _, obj = oracle.cwfilter(img, window, kind == odf.CWVMF, dist, q, level)
    n_mis, n = check_selection(idx, obj)
    assert idx.max() < window * window
    assert np.array_equal(out.reshape(-1, 3), source_pixels(img, idx, window).reshape(-1, 3))
    return n_mis, n


@pytest.mark.parametrize("window", [3, 5, 7])
@pytest.mark.parametrize("kind,dists", [(odf.CWVMF, (EXACT,)), (odf.CWDDF, (EXACT, MINIMAX, RGB))])
def test_all_levels_ragged(window, kind, dists):
    """Every level at 3x3 and 5x5; at 7x7 (25 levels) the two ends, the middle
    and two between."""
    img = synth.image_corr(61, 83, 0.2, key=30 + window)
    d = (window * window + 1) // 2
    levels = range(1, d + 1) if window < 7 else (1, 2, 7, 13, d)
    for level in levels:
        for dist in dists:
            n_mis, n = _run(img, window, kind, level, dist)
            print("  mismatch %d of %d" % (n_mis, n), flush=True)


@pytest.mark.parametrize("window", [3, 5, 7])
def test_float_and_edges(window):
    d = (window * window + 1) // 2
    for shape in ((1, 1), (1, 9), (7, 1), (29, 33)):
        img = synth.image_corr(*shape, 0.3, key=window)
        for kind in (odf.CWVMF, odf.CWDDF):
            for level in (1, 2, d):
                _run(img, window, kind, level, EXACT)
                _run(img.astype(np.float32), window, kind, level, EXACT)


@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
@pytest.mark.parametrize("window", [3, 5, 7])
def test_batch_with_zero_pixels(window, dist):
    """Three images in one call, several tiles each with ragged edges, 5 % zero
    pixels; uint8 and float32 (whose layout keeps the raw values beside the
    directions), two levels of each filter."""
    rng = np.random.default_rng(40 + 3 * window + dist)
    imgs = synth.image_corr(3 * 45, 70, 0.2, key=41).reshape(3, 45, 70, 3)
    imgs[rng.random((3, 45, 70)) < 0.05] = 0
    d = (window * window + 1) // 2
    for img in (imgs, imgs.astype(np.float32) / 255):
        for kind in (odf.CWVMF, odf.CWDDF):
            for level in (2, d // 2 + 1):
                _run(img, window, kind, level, dist)


def test_level_1_keeps_every_pixel():
    """The centre weighed n: the centre's colour wins every window (triangle
    inequality), so the output equals the input."""
    img = synth.image_uncorr(40, 50, 0.3, key=8)
    x = torch.from_numpy(img).to(DEV)
    for window in (3, 5, 7):
        for kind in (odf.CWVMF, odf.CWDDF):
            out, _ = odf.cw_filter(x, window, kind, 1, RGB)
            assert torch.equal(out, x)


def test_level_d_matches_the_plain_filters():
    """k = d weighs every member 1: CWVMF^d selects as DDF p = 1 and CWDDF^d
    as DDF p = 1/2 (the product of eq. 3), up to near-ties."""
    img = synth.image_corr(50, 70, 0.2, key=12)
    x = torch.from_numpy(img).to(DEV)
    for window in (3, 5, 7):
        d = (window * window + 1) // 2
        _, iv = odf.cw_filter(x, window, odf.CWVMF, d, EXACT)
        _, i1 = odf.filter(x, window, odf.DDF, 1.0, EXACT)
        _, ip = odf.cw_filter(x, window, odf.CWDDF, d, EXACT)
        _, ih = odf.filter(x, window, odf.DDF, 0.5, EXACT)
        for a, b in ((iv, i1), (ip, ih)):
            assert (a != b).float().mean().item() < 1e-3
