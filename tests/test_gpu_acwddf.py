"""GPU parity of the adaptive centre-weighted DDF (Section III, Experiment 2;
eq. 9 and the switching rule) against the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from paper_1009_0958_amd import synth
from parity import check_acwddf, source_pixels, window_colours

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1009_0958_amd import odf  # noqa: E402

DEV = "cuda:0"
EXACT, MINIMAX, RGB = odf.EXACT, odf.MINIMAX, odf.RGB


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def run_and_check(img, window, dist, q=4, lam=2, T=10.8, max_ambiguous=0.01):
    print("case: shape=%s w=%d dist=%d q=%d lam=%d T=%s" % (img.shape, window, dist, q, lam, T),
          flush=True)
    x = _gpu(img)
    out, idx = odf.acwddf(x, window, dist, q, lam, T)
    torch.cuda.synchronize()
    out, idx = out.cpu().numpy(), idx.cpu().numpy()
    o_out, o_idx, S, dg = oracle.acwddf(img, window, dist, q, lam, T, diag=True)
    n = window * window
    res = check_acwddf(idx, o_idx, window_colours(img, window), S, dg, n, T, max_ambiguous)
    assert idx.max() < n
    assert np.array_equal(out.reshape(-1, 3), source_pixels(img, idx, window).reshape(-1, 3))
    return res


@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
@pytest.mark.parametrize("window,lam", [(3, 1), (3, 2), (3, 3), (5, 2), (5, 11), (7, 2),
                                        (7, 23)])
def test_ragged_tiles(window, lam, dist):
    img = synth.image_corr(70, 97, 0.20, key=window * 10 + lam)
    n_mis, n_amb, n = run_and_check(img, window, dist, lam=lam)
    print("mismatch %d ambiguous %d of %d" % (n_mis, n_amb, n))


@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
@pytest.mark.parametrize("window", [3, 5, 7])
def test_sparse_zero_pixels(window, dist):
    # zero pixels among nonzero ones, also on tile boundaries: their direction is
    # (1,1,1) and their L2 terms come from the other pixel's norm
    img = synth.image_corr(70, 97, 0.15, key=40 + window + dist)
    rng = np.random.default_rng(window * 7 + dist)
    img[rng.random(img.shape[:2]) < 0.08] = 0
    img[[0, 13, 14, 29], :] = 0
    img[:, [0, 29, 30]] = 0
    # rows and columns of zeros make many windows whose selections tie in binary32
    # (e.g. several zero members); the contract still holds outside them
    n_mis, n_amb, n = run_and_check(img, window, dist, max_ambiguous=0.05)
    print("mismatch %d ambiguous %d of %d" % (n_mis, n_amb, n))


@pytest.mark.parametrize("q", [2, 3])
def test_minimax_degrees(q):
    img = synth.image_corr(48, 61, 0.2, key=q)
    run_and_check(img, 3, MINIMAX, q=q)


@pytest.mark.parametrize("T", [-1.0, 0.0, 1.0, 100.0, math.inf])
def test_thresholds(T):
    img = synth.image_corr(64, 75, 0.25, key=3)
    run_and_check(img, 3, EXACT, T=T)


@pytest.mark.parametrize("window", [3, 5, 7])
@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
def test_negative_threshold_is_ddf_product_bitwise(window, dist):
    """T < 0: every window switches to the eq. (3) selection, which the
    filter computes as DDF with p = 1/2 (same aggregates, same product)."""
    x = _gpu(synth.image_corr(80, 90, 0.2, key=7))
    _, i_acw = odf.acwddf(x, window, dist, 4, 2, -1.0)
    _, i_ddf = odf.filter(x, window, odf.DDF, 0.5, dist, 4)
    assert torch.equal(i_acw, i_ddf)
    _, i_inf = odf.acwddf(x, window, dist, 4, 2, math.inf)
    assert bool((i_inf == (window * window - 1) // 2).all())


@pytest.mark.parametrize("window", [3, 5, 7])
def test_float_inputs(window):
    img = synth.float_batch(2, 45, 70, 0.1, key=window) * 255.0
    run_and_check(img.astype(np.float32), window, EXACT)


@pytest.mark.parametrize("window", [3, 5, 7])
@pytest.mark.parametrize("shape", [(1, 1), (1, 40), (37, 1), (2, 2), (5, 5)])
def test_degenerate_sizes(window, shape):
    img = synth.image_corr(shape[0], shape[1], 0.3, key=11)
    run_and_check(img, window, EXACT)


@pytest.mark.parametrize("window", [3, 5, 7])
def test_tile_shapes_identical(window):
    x = _gpu(synth.image_corr(150, 170, 0.2, key=13))
    saved = odf.tune_get(window, odf.ACWDDF, EXACT, True)
    ref = None
    try:
        for cfg in range(4):
            try:
                odf.tune_set(window, odf.ACWDDF, EXACT, True, cfg)
            except odf.ODFError:
                assert window in (5, 7) and cfg in (0, 1)
                continue
            out, idx = odf.acwddf(x, window, EXACT)
            if ref is None:
                ref = (out, idx)
            else:
                assert torch.equal(out, ref[0]) and torch.equal(idx, ref[1])
    finally:
        odf.tune_set(window, odf.ACWDDF, EXACT, True, saved)


def test_full_size_sampled():
    """1024 x 1024 (the DDF 3x3 benchmark image) at 20000 seeded pixels."""
    img = synth.image_corr(1024, 1024, 0.20)
    x = _gpu(img)
    out, idx = odf.acwddf(x, 3, EXACT)
    idx = idx.cpu().numpy().reshape(-1)
    pix = np.random.default_rng(41).choice(1024 * 1024, 20000, replace=False)
    o_out, o_idx, S, dg = oracle.acwddf_at(img, pix, 3, EXACT)
    cols = window_colours(img, 3)[pix]
    check_acwddf(idx[pix], o_idx, cols, S, dg, 9, 10.8)
    src = source_pixels(img, idx.reshape(1024, 1024), 3).reshape(-1, 3)[pix]
    assert np.array_equal(out.cpu().numpy().reshape(-1, 3)[pix], src)


def test_hard_backward_of_acwddf_selection():
    """The one-hot backward routes through the ACWDDF index like any other."""
    img = synth.float_batch(2, 40, 50, 0.15, key=3) * 255.0
    x = _gpu(img.astype(np.float32))
    _, idx = odf.acwddf(x, 3, EXACT)
    dy = np.random.default_rng(5).standard_normal(img.shape).astype(np.float32)
    dx = odf.backward_hard(idx, _gpu(dy), 3).cpu().numpy()
    ref = oracle.backward_hard(idx.cpu().numpy(), dy.astype(np.float64), 3)
    assert np.array_equal(dx, ref.astype(np.float32))


def _sampled_window_colours(img, pix, window):
    """Member colours of the windows at flat positions pix of an (M, N, 3)
    image, (len(pix), n, 3) (replicated border), without the whole image's."""
    M, N, _ = img.shape
    h = window // 2
    r, c = np.divmod(np.asarray(pix), N)
    dy, dx = np.divmod(np.arange(window * window), window)
    rr = np.clip(r[:, None] + dy[None] - h, 0, M - 1)
    cc = np.clip(c[:, None] + dx[None] - h, 0, N - 1)
    return img[rr, cc]


@pytest.mark.parametrize("window,cfg", [(5, 2), (5, 4), (7, 2)])
def test_largest_frame_sampled(window, cfg):
    """The 7680 x 4320 frame of the benchmark's ACWDDF forms, on the tile shape
    and (5x5) the strip form that the forms' autotuner picks there: 5000 seeded
    pixels and the four corners, each pair term, against the oracle."""
    M, N = 4320, 7680
    img = synth.image_corr(M, N, 0.15, key=500)
    x = _gpu(img)
    rng = np.random.default_rng(window * 10 + cfg)
    pix = np.concatenate([rng.choice(M * N, 5000, replace=False), [0, N - 1, (M - 1) * N, M * N - 1]])
    cols = _sampled_window_colours(img, pix, window)
    for dist in (EXACT, MINIMAX, RGB):
        print("case: acwddf 7680x4320 w=%d cfg=%d dist=%d" % (window, cfg, dist), flush=True)
        saved = odf.tune_get(window, odf.ACWDDF, dist, True)
        odf.tune_set(window, odf.ACWDDF, dist, True, cfg)
        try:
            out, idx = odf.acwddf(x, window, dist)
            torch.cuda.synchronize()
        finally:
            odf.tune_set(window, odf.ACWDDF, dist, True, saved)
        gi = idx.cpu().numpy().reshape(-1)[pix]
        _, o_idx, S, dg = oracle.acwddf_at(img, pix, window, dist)
        n_mis, n_amb, n = check_acwddf(gi, o_idx, cols, S, dg, window * window, 10.8, 0.02)
        print("  mismatch %d ambiguous %d of %d" % (n_mis, n_amb, n), flush=True)
        h = window // 2
        r, c = np.divmod(pix, N)
        sr = np.clip(r + gi // window - h, 0, M - 1)
        sc = np.clip(c + gi % window - h, 0, N - 1)
        assert np.array_equal(out.cpu().numpy().reshape(-1, 3)[pix], img[sr, sc])
        del out, idx
