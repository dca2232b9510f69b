"""GPU parity at the benchmark's full sizes, in the launch forms bench.py times:
a 7680 x 4320 frame, 64 frames of 1920 x 1080 in one launch, and the 256-image
mixed batch as one planned launch.  The whole input is filtered on the GPU; the
FP64 oracle checks seeded samples of the outputs one pixel at a time."""
import numpy as np
import pytest

import oracle
from paper_1009_0958_amd import synth
from parity import check_selection

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1009_0958_amd import odf  # noqa: E402

DEV = "cuda:0"
BVDF, DDF = odf.BVDF, odf.DDF
DISTS = (odf.EXACT, odf.MINIMAX, odf.RGB)


def _sample(B, M, N, k, seed):
    """k seeded flat pixel positions plus the corners of the first and last image."""
    rng = np.random.default_rng(seed)
    corners = [0, N - 1, (M - 1) * N, M * N - 1]
    last = (B - 1) * M * N
    return np.unique(np.concatenate([rng.integers(0, B * M * N, k), corners,
                                     [last + c for c in corners]]))


def _check_sampled(imgs, out, idx, pix, window, kind, p, dist, q=4):
    """Selections at pix against the oracle (near-tie contract), outputs exact copies.
    The oracle sees each sampled pixel's window as a w x w patch of its own (border
    rows and columns replicated as the filter does), filtered at the patch centre."""
    B, M, N, _ = imgs.shape
    h = window // 2
    b, rc = np.divmod(pix, M * N)
    r, c = np.divmod(rc, N)
    off = np.arange(-h, h + 1)
    rr = np.clip(r[:, None] + off[None, :], 0, M - 1)
    cc = np.clip(c[:, None] + off[None, :], 0, N - 1)
    patches = imgs[b[:, None, None], rr[:, :, None], cc[:, None, :]]
    centre = np.arange(pix.shape[0]) * window * window + h * window + h
    _, _, _, _, oO = oracle.filter_at(patches, centre, window, kind, p, dist, q)
    g = idx.reshape(-1)[pix].astype(np.int64)
    n_mis, n = check_selection(g, oO)
    sr = np.clip(r + g // window - h, 0, M - 1)
    sc = np.clip(c + g % window - h, 0, N - 1)
    assert np.array_equal(out.reshape(-1, 3)[pix], imgs[b, sr, sc])
    return n_mis, n


def test_frame_7680x4320_sampled():
    img = synth.image_corr(4320, 7680, 0.15, key=500)[None]
    x = torch.from_numpy(img).to(DEV)
    pix = _sample(1, 4320, 7680, 6000, seed=11)
    for window, kind, p in ((3, BVDF, 0.0), (5, BVDF, 0.0), (5, DDF, 0.25), (7, BVDF, 0.0),
                            (7, DDF, 0.25)):
        for dist in DISTS:
            print("case: 7680x4320 w=%d kind=%d p=%s dist=%d" % (window, kind, p, dist), flush=True)
            out, idx = odf.filter(x, window, kind, p, dist, 4)
            n_mis, n = _check_sampled(img, out.cpu().numpy(), idx.cpu().numpy(), pix, window,
                                      kind, p, dist)
            print("  mismatch %d of %d" % (n_mis, n), flush=True)


def test_frames_64x1920x1080_one_launch_sampled():
    # 64 distinct frames: 8 generated, each shifted by a different column offset
    base = [synth.image_corr(1080, 1920, 0.15, key=600 + i) for i in range(8)]
    imgs = np.stack([np.roll(base[b % 8], 37 * b, axis=1) for b in range(64)])
    x = torch.from_numpy(imgs).to(DEV)
    pix = _sample(64, 1080, 1920, 8000, seed=12)
    for kind, p in ((BVDF, 0.0), (DDF, 0.25)):
        for dist in DISTS:
            print("case: 64x1920x1080 w=5 kind=%d dist=%d" % (kind, dist), flush=True)
            out, idx = odf.filter(x, 5, kind, p, dist, 4)
            n_mis, n = _check_sampled(imgs, out.cpu().numpy(), idx.cpu().numpy(), pix, 5, kind,
                                      p, dist)
            print("  mismatch %d of %d" % (n_mis, n), flush=True)


def test_mixed_batch_256_one_launch_sampled():
    """The benchmark's 256-image batch (windows 3 and 5, BVDF and DDF p = 1/4, eq. 8
    noise, exact angle) as one planned direct launch."""
    specs = synth.mixed_batch_specs(256)
    imgs = synth.mixed_batch_images(specs, workers=16)
    jobs = []
    for s_, im in zip(specs, imgs):
        t = torch.from_numpy(im).to(DEV)
        jobs.append(dict(img=t, out=torch.empty_like(t),
                         idx=torch.empty(t.shape[:2], dtype=torch.uint8, device=DEV),
                         window=s_["window"], kind=s_["kind"], p=s_["p"], dist=odf.EXACT, q=4))
    print("case: mixed batch of 256, %.1f Mpix" % (sum(i.shape[0] * i.shape[1] for i in imgs) / 1e6),
          flush=True)
    plan = odf.BatchPlan(jobs)
    plan.launch()
    torch.cuda.synchronize()
    total = 0
    for i, (s_, im, j) in enumerate(zip(specs, imgs, jobs)):
        M, N = im.shape[:2]
        pix = _sample(1, M, N, 200, seed=1000 + i)
        n_mis, n = _check_sampled(im[None], j["out"].cpu().numpy(), j["idx"].cpu().numpy(), pix,
                                  s_["window"], s_["kind"], s_["p"], odf.EXACT)
        total += n
    plan.close()
    print("  %d sampled pixels checked" % total, flush=True)


def _check_sampled_on_device(x, out, idx, pix, window, kind, p, dist, q=4):
    """_check_sampled for inputs too large to copy to the host: the sampled windows,
    selections and outputs are gathered on the GPU and only they are copied back."""
    B, M, N, _ = x.shape
    h = window // 2
    b, rc = np.divmod(pix, M * N)
    r, c = np.divmod(rc, N)
    off = np.arange(-h, h + 1)
    rr = np.clip(r[:, None] + off[None, :], 0, M - 1)
    cc = np.clip(c[:, None] + off[None, :], 0, N - 1)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)  # noqa: E731
    patches = x[t(b[:, None, None]), t(rr[:, :, None]), t(cc[:, None, :])].cpu().numpy()
    centre = np.arange(pix.shape[0]) * window * window + h * window + h
    _, _, _, _, oO = oracle.filter_at(patches, centre, window, kind, p, dist, q)
    g = idx.reshape(-1)[t(pix)].cpu().numpy().astype(np.int64)
    n_mis, n = check_selection(g, oO)
    sr = np.clip(r + g // window - h, 0, M - 1)
    sc = np.clip(c + g % window - h, 0, N - 1)
    got = out.reshape(-1, 3)[t(pix)].cpu().numpy()
    assert np.array_equal(got, x[t(b), t(sr), t(sc)].cpu().numpy())
    return n_mis, n


def test_largest_frame_sampled():
    """The largest frame the library accepts: 32768 x 65535 = 2^31 - 32768 pixels, so
    that byte offsets pass 2^32 (uint8) and 2^34 (float32) and the flat pixel index
    nears its int32 limit.  Random colours generated on the GPU; the last rows and
    columns are in the sample."""
    M, N = 32768, 65535
    assert M * N < 2 ** 31
    g = torch.Generator(device=DEV)
    g.manual_seed(77)
    x = torch.randint(0, 256, (1, M, N, 3), dtype=torch.uint8, device=DEV, generator=g)
    rng = np.random.default_rng(13)
    tail = np.concatenate([(M - 1) * N + rng.integers(0, N, 200),
                           rng.integers(0, M, 200) * N + N - 1])
    pix = np.unique(np.concatenate([_sample(1, M, N, 1500, seed=13), tail]))
    for window, kind, p, dist in ((3, DDF, 0.25, odf.EXACT), (5, BVDF, 0.0, odf.MINIMAX),
                                  (3, BVDF, 0.0, odf.RGB)):
        print("case: 32768x65535 u8 w=%d kind=%d p=%s dist=%d" % (window, kind, p, dist),
              flush=True)
        out, idx = odf.filter(x, window, kind, p, dist, 4)
        n_mis, n = _check_sampled_on_device(x, out, idx, pix, window, kind, p, dist)
        print("  mismatch %d of %d" % (n_mis, n), flush=True)
        del out, idx
    xf = x.float()
    del x
    print("case: 32768x65535 f32 w=3 kind=%d p=0.25 dist=%d" % (DDF, odf.EXACT), flush=True)
    out, idx = odf.filter(xf, 3, DDF, 0.25, odf.EXACT, 4)
    n_mis, n = _check_sampled_on_device(xf, out, idx, pix, 3, DDF, 0.25, odf.EXACT)
    print("  mismatch %d of %d" % (n_mis, n), flush=True)
