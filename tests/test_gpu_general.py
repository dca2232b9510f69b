"""GPU parity of the odd windows past 9x9 (11x11, 13x13, 15x15: the direct form
of the forward and the general hard backward) against the FP64 oracle,
through the C ABI."""
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


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _check(img, window, kind, p, dist):
    print("case: general %s %s w=%d kind=%d p=%s dist=%d"
          % (img.dtype, img.shape, window, kind, p, dist), flush=True)
    out, idx = odf.filter(_gpu(img), window, kind, p, dist, 4)
    out, idx = out.cpu().numpy(), idx.cpu().numpy()
    _, _, _, _, O = oracle.filter(img, window, kind, p, dist, 4, aggregates=True)
    n_mis, n = check_selection(idx, O)
    assert idx.max() < window * window
    assert np.array_equal(out.reshape(-1, 3), source_pixels(img, idx, window).reshape(-1, 3))
    return n_mis, n


@pytest.mark.parametrize("window", [11, 13, 15])
@pytest.mark.parametrize("kind,p", [(BVDF, 0.0), (DDF, 0.25), (DDF, 0.5), (DDF, 0.3)])
@pytest.mark.parametrize("u8", [True, False])
def test_forward_matches_oracle(window, kind, p, u8):
    """Two images of several 8 x 8 window blocks with ragged edges both ways,
    5 % zero pixels, every pair term."""
    rng = np.random.default_rng(window * 10 + kind)
    img = synth.image_corr(2 * 21, 27, 0.2, key=window + kind).reshape(2, 21, 27, 3)
    img[rng.random((2, 21, 27)) < 0.05] = 0
    x = img if u8 else (img.astype(np.float32) / 255.0).astype(np.float32)
    for dist in (EXACT, MINIMAX, RGB):
        n_mis, n = _check(x, window, kind, p, dist)
        print("  mismatch %d of %d" % (n_mis, n), flush=True)


@pytest.mark.parametrize("window", [11, 15])
def test_degenerate_shapes(window):
    for shape in ((1, 1), (1, 40), (30, 1), (5, 5), (9, 17)):
        img = synth.image_corr(*shape, 0.3, key=window)
        _check(img, window, DDF, 0.25, EXACT)
        _check(img.astype(np.float32), window, BVDF, 0.0, RGB)


@pytest.mark.parametrize("window", [11, 13, 15])
def test_exact_ties_go_to_the_lowest_index(window):
    """A constant image ties every member (index 0); a BVDF window of collinear
    uint8 colours ties every member too (one canonical direction)."""
    const = np.full((1, 20, 30, 3), (90, 30, 150), np.uint8)
    for kind, p in ((BVDF, 0.0), (DDF, 0.25)):
        for dist in (EXACT, MINIMAX, RGB):
            out, idx = odf.filter(_gpu(const), window, kind, p, dist)
            assert bool((idx == 0).all()) and torch.equal(out, _gpu(const))
    rng = np.random.default_rng(window)
    scale = rng.integers(1, 9, (1, 20, 30, 1)).astype(np.uint8)
    coll = scale * np.array([3, 7, 11], np.uint8)
    _, idx = odf.filter(_gpu(coll), window, BVDF, 0.0, EXACT)
    assert bool((idx == 0).all())


@pytest.mark.parametrize("window", [11, 13, 15])
def test_backward_hard_matches_oracle_bitwise(window):
    """The general hard backward against the oracle's raster-order binary64
    sums, on the filter's own selections and with 10 % foreign indices
    (>= n, which route nothing)."""
    print("case: general hard bwd w=%d" % window, flush=True)
    B, M, N = 2, 23, 70
    x = synth.float_batch(B, M, N, 0.1, key=window)
    _, idx = odf.filter(_gpu(x), window, DDF, 0.25)
    idx = idx.cpu().numpy()
    rng = np.random.default_rng(window)
    dy = rng.standard_normal(x.shape).astype(np.float32)
    dx = odf.backward_hard(_gpu(idx), _gpu(dy), window).cpu().numpy()
    ref = oracle.backward_hard(idx, dy.astype(np.float64), window)
    assert np.array_equal(dx, ref.astype(np.float32))
    bad = rng.random(idx.shape) < 0.1
    idx_bad = idx.copy()
    idx_bad[bad] = rng.integers(window * window, 256, int(bad.sum()))
    dx = odf.backward_hard(_gpu(idx_bad), _gpu(dy), window).cpu().numpy()
    dy0 = dy.astype(np.float64)
    dy0[bad] = 0.0
    assert np.array_equal(dx, oracle.backward_hard(idx, dy0, window).astype(np.float32))


def test_hard_filter_autograd_15x15():
    x = _gpu(synth.float_batch(1, 19, 26, 0.15, key=15)).requires_grad_(True)
    y, idx = odf.hard_filter(x, 15, DDF, 0.5)
    w = torch.randn_like(y)
    (y * w).sum().backward()
    ref = oracle.backward_hard(idx.cpu().numpy(), w.cpu().numpy().astype(np.float64), 15)
    assert np.array_equal(x.grad.cpu().numpy(), ref.astype(np.float32))


def test_sampled_1080p():
    """One 1920 x 1080 uint8 frame at 11 x 11 (DDF p = 1/4, exact): 3000
    seeded pixels and the four corners against the oracle's per-pixel form."""
    img = synth.image_corr(1080, 1920, 0.15, key=11)
    out, idx = odf.filter(_gpu(img), 11, DDF, 0.25, EXACT)
    out, idx = out.cpu().numpy(), idx.cpu().numpy()
    rng = np.random.default_rng(1080)
    M, N = 1080, 1920
    pix = np.concatenate([rng.permutation(M * N)[:3000], [0, N - 1, (M - 1) * N, M * N - 1]])
    _, _, _, _, O = oracle.filter_at(img, pix, 11, DDF, 0.25, EXACT)
    n_mis, n = check_selection(idx.reshape(-1)[pix], O)
    print("1080p 11x11: mismatch %d of %d" % (n_mis, n), flush=True)
    src = source_pixels(img, idx, 11).reshape(-1, 3)
    assert np.array_equal(out.reshape(-1, 3), src)


@pytest.mark.parametrize("window", [9, 11, 15])
@pytest.mark.parametrize("u8", [True, False])
def test_acwddf_direct_form(window, u8):
    """ACWDDF (lambda = 2, T = 10.8) at 9x9 to 15x15 on the direct form, every
    pair term, against the oracle's selections and switching statistic (the
    selection may differ only where binary32 can change a level's argmin or
    the side of T)."""
    from parity import check_acwddf, window_colours
    img = synth.image_corr(2 * 19, 26, 0.2, key=window).reshape(2, 19, 26, 3)
    x = img if u8 else img.astype(np.float32)
    n = window * window
    for dist in (EXACT, MINIMAX, RGB):
        print("case: general acwddf %s w=%d dist=%d" % (x.dtype, window, dist), flush=True)
        out, idx = odf.acwddf(_gpu(x), window, dist, 4, 2, 10.8)
        out, idx = out.cpu().numpy(), idx.cpu().numpy()
        _, o_idx, S, dg = oracle.acwddf(x, window, dist, 4, 2, 10.8, diag=True)
        n_mis, n_amb, n_tot = check_acwddf(idx, o_idx, window_colours(x, window), S, dg, n,
                                           10.8, 0.05)
        print("  mismatch %d ambiguous %d of %d" % (n_mis, n_amb, n_tot), flush=True)
        assert np.array_equal(out.reshape(-1, 3), source_pixels(x, idx, window).reshape(-1, 3))


@pytest.mark.parametrize("window", [9, 13])
@pytest.mark.parametrize("u8", [True, False])
def test_centre_weighted_direct_form(window, u8):
    """CWVMF^k and CWDDF^k at 9x9 and 13x13 on the direct form: levels 1, 2,
    a middle one and d, against the oracle's objectives."""
    img = synth.image_corr(2 * 17, 23, 0.2, key=30 + window).reshape(2, 17, 23, 3)
    x = img if u8 else img.astype(np.float32) / 255
    d = (window * window + 1) // 2
    for kind, dists in ((odf.CWVMF, (EXACT,)), (odf.CWDDF, (EXACT, MINIMAX, RGB))):
        for level in (1, 2, d // 2, d):
            for dist in dists:
                print("case: general cw %s w=%d kind=%d level=%d dist=%d"
                      % (x.dtype, window, kind, level, dist), flush=True)
                out, idx = odf.cw_filter(_gpu(x), window, kind, level, dist, 4)
                out, idx = out.cpu().numpy(), idx.cpu().numpy()
                _, _, obj = oracle.cwfilter(x, window, kind == odf.CWVMF, dist, 4, level)
                check_selection(idx, obj)
                assert np.array_equal(out.reshape(-1, 3),
                                      source_pixels(x, idx, window).reshape(-1, 3))


def test_centre_weighted_extremes_direct_form():
    """Level 1 keeps every pixel (the centre weighed n wins by the triangle
    inequality) and ACWDDF with T = +inf keeps every centre, at 11x11."""
    img = synth.image_uncorr(20, 27, 0.3, key=8)
    x = _gpu(img)
    for kind in (odf.CWVMF, odf.CWDDF):
        out, _ = odf.cw_filter(x, 11, kind, 1, RGB)
        assert torch.equal(out, x)
    _, idx = odf.acwddf(x, 11, EXACT, 4, 2, float("inf"))
    assert bool((idx == 60).all())
