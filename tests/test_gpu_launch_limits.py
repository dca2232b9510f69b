"""GPU parity at shapes whose workgroup counts pass a single grid dimension's
limits: more than 65535 images in one call, an image more than 65535 tiles tall,
and more than 65535 one-tile jobs in one batch.  Every kernel numbers its tiles
over a flat two-dimensional grid, so these shapes run like any other; each case
is checked in full against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1009_0958_amd import synth
from parity import (check_acwddf, check_selection, check_soft, soft_bounds, source_pixels,
                    window_colours)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1009_0958_amd import odf  # noqa: E402

DEV = "cuda:0"
BVDF, DDF = odf.BVDF, odf.DDF
EXACT, MINIMAX, RGB = odf.EXACT, odf.MINIMAX, odf.RGB


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _forward(img, window, kind, p, dist):
    print("case: forward %s w=%d kind=%d p=%s dist=%d" % (img.shape, window, kind, p, dist),
          flush=True)
    out, idx = odf.filter(_gpu(img), window, kind, p, dist, 4)
    out, idx = out.cpu().numpy(), idx.cpu().numpy()
    _, _, _, _, oO = oracle.filter(img, window, kind, p, dist, 4, aggregates=True)
    n_mis, n = check_selection(idx, oO)
    assert np.array_equal(out.reshape(-1, 3), source_pixels(img, idx, window).reshape(-1, 3))
    print("  mismatch %d of %d" % (n_mis, n), flush=True)
    return idx


def _gradients(x, idx, window, kind, p, tau, seed):
    """Hard backward (bitwise) and softmin forward and backward (error budget)."""
    print("case: gradients %s w=%d" % (x.shape, window), flush=True)
    dy = np.random.default_rng(seed).standard_normal(x.shape).astype(np.float32)
    dx = odf.backward_hard(_gpu(idx), _gpu(dy), window).cpu().numpy()
    assert np.array_equal(dx, oracle.backward_hard(idx, dy.astype(np.float64), window)
                          .astype(np.float32))
    y = odf.softmin_forward(_gpu(x), window, kind, p, tau).cpu().numpy()
    ref_y = oracle.softmin_fwd(x, window, kind, p, tau)
    dx = odf.softmin_backward(_gpu(x), _gpu(dy), window, kind, p, tau).cpu().numpy()
    ref = oracle.softmin_bwd(x, dy.astype(np.float64), window, kind, p, tau)
    omega = oracle.filter(x, window, kind, p, EXACT, aggregates=True)[4]
    check_soft(y, ref_y, dx, ref, soft_bounds(x, omega, window, tau, np.abs(ref).max()),
               "softmin %s" % (x.shape,))


def _acwddf(img, window):
    print("case: acwddf %s w=%d" % (img.shape, window), flush=True)
    out, idx = odf.acwddf(_gpu(img), window, EXACT, 4, 2, 10.8)
    out, idx = out.cpu().numpy(), idx.cpu().numpy()
    _, o_idx, S, dg = oracle.acwddf(img, window, EXACT, 4, 2, 10.8, diag=True)
    check_acwddf(idx, o_idx, window_colours(img, window), S, dg, window * window, 10.8, 0.02)
    assert np.array_equal(out.reshape(-1, 3), source_pixels(img, idx, window).reshape(-1, 3))


def test_more_than_65535_images():
    """70000 images of 3 x 4 pixels in one call: 70000 workgroups along what was the
    image dimension of the grid."""
    B, M, N = 70000, 3, 4
    imgs = synth.image_corr(B * M, N, 0.15, key=70).reshape(B, M, N, 3)
    idx = _forward(imgs, 3, DDF, 0.25, EXACT)
    _forward(imgs, 5, BVDF, 0.0, MINIMAX)
    keep = odf.tune_get(5, DDF, EXACT, True)
    try:
        odf.tune_set(5, DDF, EXACT, True, odf.STRIP)  # the strip form: one strip per image
        _forward(imgs, 5, DDF, 0.25, EXACT)
    finally:
        odf.tune_set(5, DDF, EXACT, True, keep)
    _acwddf(imgs, 3)
    _gradients(imgs.astype(np.float32) / 255, idx, 3, DDF, 0.25, 0.1, seed=70)


def test_taller_than_65535_tiles():
    """A 1,000,000 x 2 frame, each kernel on a tile of at most 14 output rows, so that
    every grid has more than 65535 tile rows: 83334 for the 5 x 5 forward (32 x 16
    extended tile), 71429 and 166667 for the 3 x 3 forward on the 32 x 16 and 64 x 8
    tiles, 71429 for the softmin, 125000 for the hard backward (64 x 8 tiles) and 250000
    for the softmin's combine pass."""
    M, N = 1_000_000, 2
    img = synth.image_corr(M, N, 0.15, key=71)
    _forward(img, 5, BVDF, 0.0, EXACT)
    keep = [odf.tune_get(3, DDF, d, True) for d in (EXACT, RGB)]
    try:
        odf.tune_set(3, DDF, RGB, True, 2)    # 32 x 16 extended tile, 14 output rows
        odf.tune_set(3, DDF, EXACT, True, 3)  # 64 x 8, 6 output rows
        idx = _forward(img, 3, DDF, 0.25, RGB)
        _forward(img, 3, DDF, 0.25, EXACT)
    finally:
        odf.tune_set(3, DDF, EXACT, True, keep[0])
        odf.tune_set(3, DDF, RGB, True, keep[1])
    _gradients(img.astype(np.float32) / 255, idx, 3, DDF, 0.25, 0.1, seed=71)


def test_batch_of_70000_jobs():
    """70000 one-tile jobs (views into one buffer) in one direct batch launch, so
    the direct kernel's grid passes 65535 workgroups in one group."""
    B, M, N = 70000, 5, 6
    imgs = synth.image_corr(B * M, N, 0.15, key=72).reshape(B, M, N, 3)
    x = _gpu(imgs)
    out = torch.empty_like(x)
    idx = torch.empty((B, M, N), dtype=torch.uint8, device=DEV)
    jobs = [dict(img=x[b], out=out[b], idx=idx[b], window=3, kind=DDF, p=0.25, dist=EXACT, q=4)
            for b in range(B)]
    print("case: batch of %d jobs" % B, flush=True)
    plan = odf.BatchPlan(jobs)
    assert plan.info()["tiles"][3 * 1 + EXACT] == B
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    out, idx = out.cpu().numpy(), idx.cpu().numpy()
    _, _, _, _, oO = oracle.filter(imgs, 3, DDF, 0.25, EXACT, 4, aggregates=True)
    n_mis, n = check_selection(idx, oO)
    assert np.array_equal(out.reshape(-1, 3), source_pixels(imgs, idx, 3).reshape(-1, 3))
    print("  mismatch %d of %d" % (n_mis, n), flush=True)
