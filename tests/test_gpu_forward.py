"""GPU parity of the forward filter (HIP, through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1009_0958_amd import synth
from parity import AGG_RTOL, check_aggregates, check_selection, source_pixels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1009_0958_amd import odf  # noqa: E402

DEV = "cuda:0"
BVDF, DDF = odf.BVDF, odf.DDF
EXACT, MINIMAX, RGB = odf.EXACT, odf.MINIMAX, odf.RGB


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def run_and_check(img, window, kind, p, dist, q=4, aggregates=True, agg_rtol=AGG_RTOL):
    """Full-image parity: selections, output copies and aggregates."""
    print("case: shape=%s w=%d kind=%d p=%s dist=%d q=%d" % (img.shape, window, kind, p, dist, q),
          flush=True)
    x = _gpu(img)
    out, idx = odf.filter(x, window, kind, p, dist, q)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    idx = idx.cpu().numpy()
    o_out, o_idx, oA, oD, oO = oracle.filter(img, window, kind, p, dist, q, aggregates=True)
    n_mis, n = check_selection(idx, oO)
    assert np.array_equal(out.reshape(-1, 3),
                          source_pixels(img, idx, window).reshape(-1, 3))
    assert idx.max() < window * window
    if aggregates:
        A, D, O = (t.cpu().numpy() for t in odf.aggregates(x, window, kind, p, dist, q))
        check_aggregates(A, oA, agg_rtol, name="A")
        if kind == DDF:
            check_aggregates(D, oD, name="D")
        check_aggregates(O, oO, agg_rtol, name="Omega")
    return n_mis, n


@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
def test_bvdf3_256_uncorrelated(dist):
    img = synth.image_uncorr(256, 256, 0.10)
    n_mis, n = run_and_check(img, 3, BVDF, 0.0, dist)
    print("mismatch %d / %d" % (n_mis, n))


@pytest.mark.parametrize("p", [0.25, 0.5])
@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
def test_ddf3_correlated_crop(p, dist):
    img = synth.image_corr(200, 172, 0.20)
    run_and_check(img, 3, DDF, p, dist)


@pytest.mark.parametrize("kind,p", [(BVDF, 0.0), (DDF, 0.25), (DDF, 0.5)])
@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
def test_window5_ragged(kind, p, dist):
    img = synth.image_corr(70, 93, 0.15, key=5)
    run_and_check(img, 5, kind, p, dist)


@pytest.mark.parametrize("kind,p", [(BVDF, 0.0), (DDF, 0.25), (DDF, 0.5)])
@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
def test_window7_ragged(kind, p, dist):
    img = synth.image_corr(45, 71, 0.15, key=7)
    run_and_check(img, 7, kind, p, dist)


@pytest.mark.parametrize("q", [2, 3, 4])
@pytest.mark.parametrize("window", [3, 5])
def test_minimax_degrees(q, window):
    img = synth.image_corr(61, 67, 0.2, key=q)
    run_and_check(img, window, DDF, 0.25, MINIMAX, q)
    run_and_check(img, window, BVDF, 0.0, MINIMAX, q)


@pytest.mark.parametrize("window", [3, 5, 7])
@pytest.mark.parametrize("kind,p", [(BVDF, 0.0), (DDF, 0.25), (DDF, 1.0), (DDF, 0.0)])
def test_float_inputs_exact(window, kind, p):
    img = synth.float_batch(2, 45, 70, 0.1, key=window)
    run_and_check(img, window, kind, p, EXACT)


@pytest.mark.parametrize("window", [3, 5, 7])
@pytest.mark.parametrize("dist", [MINIMAX, RGB])
@pytest.mark.parametrize("kind,p", [(BVDF, 0.0), (DDF, 0.25)])
def test_float_inputs_minimax_rgb(window, dist, kind, p):
    """float32 inputs (non-negative, as minimax and the chromaticity term need)
    with the two fast pair terms; every window size, both kinds: selections to
    the near-tie band, aggregates within 1e-5 relative (the chromaticity
    numerators and cross products of float pixels are formed in binary64)."""
    img = synth.float_batch(2, 41, 66, 0.1, key=40 + window + dist)
    run_and_check(img, window, kind, p, dist)


@pytest.mark.parametrize("window", [3, 5])
@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
@pytest.mark.parametrize("kind,p", [(BVDF, 0.0), (DDF, 0.25)])
def test_float_nearly_parallel(window, dist, kind, p):
    """Nearly parallel float colours (a grey level with perturbations of 1e-3,
    angles and chromaticity distances of ~1e-3): the cross products and
    chromaticity numerators cancel to ~1e-3 of their operands, where binary32
    differences of rounded products would leave ~3e-5 relative error per term;
    aggregates must still be within 1e-5 of the oracle."""
    rng = np.random.default_rng(61 + window + 3 * dist)
    img = (0.5 + rng.uniform(-1e-3, 1e-3, (2, 37, 45, 3))).astype(np.float32)
    img[:, 5:9, 7:12] *= np.float32(1.75)  # collinear block: same angles, other L2 terms
    run_and_check(img, window, kind, p, dist)


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (9, 1), (2, 3), (30, 30), (31, 29), (28, 28),
                                   (29, 57), (5, 200)])
@pytest.mark.parametrize("window", [3, 5, 7])
def test_edge_shapes(shape, window):
    rng = np.random.default_rng(sum(shape) * window)
    img = rng.integers(0, 256, shape + (3,)).astype(np.uint8)
    img[rng.random(shape) < 0.2] = 0
    run_and_check(img, window, DDF, 0.25, EXACT)
    run_and_check(img, window, BVDF, 0.0, RGB)


def test_batch_of_three():
    imgs = np.stack([synth.image_corr(40, 52, 0.2, key=k) for k in range(3)])
    run_and_check(imgs, 3, DDF, 0.5, EXACT)
    run_and_check(imgs, 5, BVDF, 0.0, MINIMAX)


@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
def test_degenerate_images(dist):
    const = np.full((33, 41, 3), (120, 40, 200), np.uint8)
    zero = np.zeros((17, 19, 3), np.uint8)
    ramp = np.repeat(np.repeat(np.arange(10, 10 + 12 * 20, 12, dtype=np.uint8)[:, None], 20, 1)
                     [..., None], 3, 2)
    for img in (const, zero, ramp):
        for kind, p in ((BVDF, 0.0), (DDF, 0.5)):
            x = _gpu(img)
            out, idx = odf.filter(x, 3, kind, p, dist)
            out, idx = out.cpu().numpy(), idx.cpu().numpy()
            # a gray ramp has all angles 0 (exact); minimax gives every pair a_0 > 0
            # and DDF then orders by D, so only the exact ramp must select u = 0
            if img is not ramp or (dist == EXACT) or (kind == BVDF and dist != RGB):
                assert np.all(idx == 0), (dist, kind)
            run_and_check(img, 3, kind, p, dist)


def _sparse_zeros(M, N, key):
    """A smooth image with 8 % of its pixels (0, 0, 0), whole rows and columns of zeros on
    and next to tile boundaries, and a zero corner."""
    img = synth.image_corr(M, N, 0.15, key=key)
    rng = np.random.default_rng(key)
    img[rng.random((M, N)) < 0.08] = 0
    img[[0, 13, 14, 29, 30], :] = 0
    img[:, [0, 29, 30, 31]] = 0
    img[-3:, -4:] = 0
    return img


@pytest.mark.parametrize("u8", [True, False])
@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
@pytest.mark.parametrize("window", [3, 5, 7])
def test_sparse_zero_pixels(window, dist, u8):
    # the zero pixel's direction (1,1,1) and value 0 next to nonzero neighbours: the
    # uint8 layout marks it by the sign of its stored norm and takes its L2 terms from
    # the other pixel's norm; the float layout meets it through a zero norm
    img = _sparse_zeros(70, 97, key=window * 3 + dist)
    if not u8:
        img = img.astype(np.float32) / 255
    for kind, p in ((BVDF, 0.0), (DDF, 0.25), (DDF, 1.0)):
        run_and_check(img, window, kind, p, dist, aggregates=window < 7)


# 3x3 pattern whose colour X (twice) minimises every objective of a window holding it
_X = (100, 80, 60)
_PATTERN = np.array([[(120, 70, 75), (85, 90, 50), _X], [(110, 95, 52), (92, 66, 70), (104, 71, 49)],
                     [_X, (96, 88, 66), (108, 84, 58)]], np.uint8)


@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
@pytest.mark.parametrize("u8", [True, False])
def test_duplicate_colours_tie_exactly(dist, u8):
    # Tiled with period 3, every interior 3x3 window holds the pattern's nine cells, so the
    # two members of colour X tie in every objective; the filter must take the lower index.
    # The member's term with itself (a per-variant constant) and its term with an equal
    # colour (a pair evaluation) have to agree bit for bit for the tie to be exact.
    M, N = 70, 97
    img = np.tile(_PATTERN, (M // 3 + 1, N // 3 + 1, 1))[:M, :N]
    x = _gpu(img if u8 else img.astype(np.float32))
    for kind, p in ((BVDF, 0.0), (DDF, 0.25), (DDF, 0.5)):
        _, idx = odf.filter(x, 3, kind, p, dist)
        idx = idx.cpu().numpy()
        for r in range(1, M - 1):
            for c in range(1, N - 1):
                win = img[r - 1:r + 2, c - 1:c + 2].reshape(9, 3)
                want = int(np.flatnonzero((win == _X).all(1))[0])
                assert idx[r, c] == want, (dist, u8, kind, p, r, c, idx[r, c], want)


@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
def test_lone_impulse_never_selected(dist):
    img = np.full((21, 23, 3), (100, 50, 20), np.uint8)
    img[10, 11] = (20, 200, 40)
    for window in (3, 5):
        for kind, p in ((BVDF, 0.0), (DDF, 0.25)):
            out, _ = odf.filter(_gpu(img), window, kind, p, dist)
            assert np.all(out.cpu().numpy() == np.array([100, 50, 20], np.uint8))


def test_scaling_by_two_bit_exact():
    img = (synth.image_corr(96, 80, 0.2, key=9) // 2).astype(np.uint8)
    for window in (3, 5):
        for dist in (EXACT, MINIMAX, RGB):
            _, i1 = odf.filter(_gpu(img), window, BVDF, 0.0, dist)
            _, i2 = odf.filter(_gpu(img * 2), window, BVDF, 0.0, dist)
            assert torch.equal(i1, i2)


def test_float_power_of_two_scaling_bit_exact():
    img = synth.float_batch(1, 50, 60, 0.1, key=3)
    for kind, p in ((BVDF, 0.0), (DDF, 0.25)):
        _, i1 = odf.filter(_gpu(img), 5, kind, p, EXACT)
        _, i2 = odf.filter(_gpu(img * 8.0), 5, kind, p, EXACT)
        if kind == BVDF:
            assert torch.equal(i1, i2)
        else:  # D scales by 8: the objective gains a constant log2 term
            assert (i1 != i2).float().mean().item() < 1e-3


@pytest.mark.parametrize("scale_exp", [61, -30])
def test_float_domain_edges(scale_exp):
    """Near both ends of the documented float32 domain (values up to 2^61; and
    scaled by 2^-30, where the L2 distances of distinct pixels stay far above the
    2^-63 below which their squares turn subnormal) the filter still meets the
    parity contract: selections to the near-tie band, A, D and Omega within
    1e-5 of the oracle."""
    img = synth.float_batch(1, 34, 41, 0.1, key=30) * np.float32(2.0 ** scale_exp)
    for window, kind, p, dist in ((5, DDF, 0.25, EXACT), (3, DDF, 0.5, EXACT), (3, DDF, 0.3, EXACT),
                                  (3, DDF, 1.0, MINIMAX), (5, DDF, 0.25, RGB), (3, BVDF, 0.0, EXACT)):
        run_and_check(img, window, kind, p, dist)


def test_caller_outputs_are_used_and_returned():
    img = synth.image_corr(33, 40, 0.2, key=3)
    x = _gpu(img)
    ref_o, ref_i = odf.filter(x, 3, DDF, 0.25, EXACT)
    out = torch.empty_like(x)
    idx = torch.empty((33, 40), dtype=torch.uint8, device=DEV)
    o, i = odf.filter(x, 3, DDF, 0.25, EXACT, out=out, idx=idx)
    assert o is out and i is idx
    torch.cuda.synchronize()
    assert torch.equal(out, ref_o) and torch.equal(idx, ref_i)
    xb = x[None]
    ob = torch.empty_like(xb)
    o, i = odf.acwddf(xb, 3, EXACT, 4, 2, 10.8, out=ob, return_idx=False)
    assert o is ob and i is None
    for bad in (dict(out=out[:, :20]), dict(out=torch.empty_like(x, dtype=torch.float32)),
                dict(idx=idx[:20]), dict(out=torch.empty((1, 33, 40, 3), dtype=torch.uint8))):
        with pytest.raises(ValueError):
            odf.filter(x, 3, DDF, 0.25, EXACT, **bad)


def test_deterministic_repeat():
    img = _gpu(synth.image_corr(300, 310, 0.2, key=11))
    for window, kind, p, dist in ((3, DDF, 0.25, EXACT), (5, BVDF, 0.0, MINIMAX),
                                  (5, DDF, 0.5, RGB)):
        o1, i1 = odf.filter(img, window, kind, p, dist)
        o2, i2 = odf.filter(img, window, kind, p, dist)
        assert torch.equal(o1, o2) and torch.equal(i1, i2)


@pytest.mark.parametrize("window,kind,p,dist", [
    (3, DDF, 0.25, EXACT), (3, DDF, 0.5, EXACT), (3, DDF, 0.25, MINIMAX), (3, DDF, 0.5, RGB),
    (5, BVDF, 0.0, EXACT), (5, DDF, 0.25, EXACT), (5, DDF, 0.25, MINIMAX), (5, DDF, 0.25, RGB),
    (7, BVDF, 0.0, EXACT), (7, DDF, 0.25, EXACT)])
def test_full_size_sampled(window, kind, p, dist):
    """1024 x 1024 with correlated noise 0.20: the whole image on the GPU,
    checked on 20 000 seeded sample pixels (plus the four corners) by the oracle."""
    img = synth.image_corr(1024, 1024, 0.20)
    x = _gpu(img)
    out, idx = odf.filter(x, window, kind, p, dist)
    out, idx = out.cpu().numpy(), idx.cpu().numpy()
    rng = np.random.default_rng(77)
    M, N = img.shape[:2]
    pix = np.unique(np.concatenate([rng.integers(0, M * N, 20000),
                                    [0, N - 1, (M - 1) * N, M * N - 1]]))
    _, o_idx, _, _, oO = oracle.filter_at(img, pix, window, kind, p, dist)
    check_selection(idx.reshape(-1)[pix], oO)
    src = source_pixels(img, idx, window).reshape(-1, 3)
    assert np.array_equal(out.reshape(-1, 3), src)


@pytest.mark.parametrize("kind,p", [(BVDF, 0.0), (DDF, 0.25)])
def test_window7_tile_shapes_identical(kind, p):
    x = _gpu(synth.image_corr(100, 130, 0.2, key=17))
    saved = odf.tune_get(7, kind, EXACT, True)
    try:
        odf.tune_set(7, kind, EXACT, True, 2)
        a = odf.filter(x, 7, kind, p, EXACT)
        odf.tune_set(7, kind, EXACT, True, 3)
        b = odf.filter(x, 7, kind, p, EXACT)
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    finally:
        odf.tune_set(7, kind, EXACT, True, saved)


def _collinear_image(M, N, seed):
    """Mostly positive multiples of (1, 2, 3) and of (4, 1, 0) at different
    brightness (windows whose minimum is shared by collinear colours), with
    other colours and zero pixels scattered in."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, 64, (M, N))
    base = np.where((rng.random((M, N)) < 0.5)[..., None], np.array([1, 2, 3]), np.array([4, 1, 0]))
    img = (k[..., None] * base).astype(np.uint8)
    other = rng.random((M, N)) < 0.2
    img[other] = rng.integers(0, 256, (int(other.sum()), 3))
    img[rng.random((M, N)) < 0.02] = 0
    return img


@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
@pytest.mark.parametrize("window", [3, 5, 7, 9])
def test_bvdf_collinear_colours_select_lowest_index(window, dist):
    """BVDF on uint8 pixels takes the canonical direction x / gcd(x), as the
    oracle does: members that are multiples of one colour tie bit for bit and
    the lowest index wins, so the GPU's index equals the oracle's at every pixel
    whose minimum is shared by collinear colours (and elsewhere up to near-ties
    between different directions); per-image and batched launches agree."""
    img = _collinear_image(*((70, 97) if window < 9 else (40, 50)), 80 + window + dist)
    n_mis, n = run_and_check(img, window, BVDF, 0.0, dist, aggregates=(window < 7))
    _, idx = odf.filter(_gpu(img), window, BVDF, 0.0, dist)
    idx = idx.cpu().numpy()
    _, o_idx, _, _, O = oracle.filter(img, window, BVDF, 0.0, dist, aggregates=True)
    M, N = idx.shape
    h = window // 2
    rr = np.clip(np.arange(M)[:, None, None] + np.arange(window * window)[None, None, :] // window - h,
                 0, M - 1)
    cc = np.clip(np.arange(N)[None, :, None] + np.arange(window * window)[None, None, :] % window - h,
                 0, N - 1)
    mem = img[rr, cc].astype(np.int64)  # M, N, n, 3
    omin = O.min(-1, keepdims=True)
    tied = O == omin
    first = mem[np.arange(M)[:, None], np.arange(N)[None, :], o_idx.astype(np.int64)]
    coll = np.all(np.cross(mem, first[:, :, None, :]) == 0, axis=-1)
    only_collinear = np.all(~tied | coll, axis=-1) & (tied.sum(-1) > 1)
    assert only_collinear.sum() > 50
    assert np.array_equal(idx[only_collinear], o_idx[only_collinear])
    if window >= 7:
        return  # the batch takes windows 3 and 5
    # the batched launch (two copies, one job each) gives the same indices
    x = _gpu(img)
    jobs = [dict(img=x, out=torch.empty_like(x), idx=torch.empty((M, N), dtype=torch.uint8,
                                                                  device=DEV),
                 window=window, kind=BVDF, p=0.0, dist=dist, q=4) for _ in range(2)]
    plan = odf.BatchPlan(jobs)
    plan.launch()
    torch.cuda.synchronize()
    for j in jobs:
        assert np.array_equal(j["idx"].cpu().numpy(), idx)
    plan.close()


@pytest.mark.parametrize("u8", [True, False])
@pytest.mark.parametrize("dist", [EXACT, MINIMAX, RGB])
@pytest.mark.parametrize("kind,p", [(BVDF, 0.0), (DDF, 0.25)])
def test_window9(kind, p, dist, u8):
    """9 x 9 windows (h = 4, one 32 x 16 extended tile of 24 x 8 output pixels):
    a ragged image of 3 x 5 tiles with zero pixels, uint8 and float32, against
    the oracle: selections to the near-tie band, copies, aggregates."""
    img = _sparse_zeros(36, 52, key=90 + dist)
    if not u8:
        img = img.astype(np.float32) / 255
    run_and_check(img, 9, kind, p, dist)


@pytest.mark.parametrize("shape", [(1, 1), (2, 3), (9, 1), (5, 30), (17, 25)])
def test_window9_edge_shapes(shape):
    rng = np.random.default_rng(sum(shape) + 9)
    img = rng.integers(0, 256, shape + (3,)).astype(np.uint8)
    img[rng.random(shape) < 0.2] = 0
    run_and_check(img, 9, DDF, 0.25, EXACT)
    run_and_check(img, 9, BVDF, 0.0, RGB)

