"""GPU tests of the batched launch, its graph capture and the tile-shape
autotuners (per image and per batch group): results must be bitwise those of
the per-image filter (and so of the oracle up to near-ties), whatever the tile
shape or schedule."""
import numpy as np
import pytest

import oracle
from paper_1009_0958_amd import synth
from parity import check_selection

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1009_0958_amd import odf  # noqa: E402

DEV = "cuda:0"


def _mixed_jobs(count, seed, max_side=160):
    rng = np.random.default_rng(seed)
    jobs, refs = [], []
    for i in range(count):
        M = int(rng.integers(1, max_side))
        N = int(rng.integers(1, max_side))
        img = synth.noise_eq8(synth.smooth_image(M, N, synth.rng_for(9, seed, i)),
                              float(rng.uniform(0.05, 0.3)), rng)
        job = dict(img=torch.from_numpy(img).to(DEV),
                   out=torch.empty((M, N, 3), dtype=torch.uint8, device=DEV),
                   idx=torch.empty((M, N), dtype=torch.uint8, device=DEV),
                   window=int(rng.choice([3, 5, 7, 9])), kind=int(rng.integers(0, 2)),
                   dist=int(rng.integers(0, 3)), q=int(rng.integers(2, 5)),
                   p=float(rng.choice([0.0, 0.25, 0.5, 1.0])))
        jobs.append(job)
        refs.append(img)
    return jobs, refs


def _per_image(job):
    return odf.filter(job["img"], job["window"], job["kind"], job["p"], job["dist"], job["q"])


@pytest.mark.parametrize("cfg", [0, 1, 2, 3, 4, 5])
def test_batch_equals_per_image_and_oracle(cfg):
    """Every group on config cfg (the batch tuning table set for all eight): a
    tile shape, or the strip form (4: 8 bands per strip, 5: 3 bands); groups
    that do not offer cfg (7x7: the 1024-thread shapes; 9x9: all but shape 2
    and, for BVDF, the strips) stay on shape 2 there."""
    jobs, imgs = _mixed_jobs(40, 1)
    assert {j["window"] for j in jobs} == {3, 5, 7, 9}
    keep = {(w, k): odf.batch_tune_get(w, k) for w in (3, 5, 7, 9) for k in (0, 1)}
    expect = []
    try:
        for (w, k) in keep:
            try:
                odf.batch_tune_set(w, k, cfg)
            except odf.ODFError:
                assert w >= 7
                odf.batch_tune_set(w, k, 2)
            expect.append(odf.batch_tune_get(w, k))
        plan = odf.BatchPlan(jobs)
    finally:
        for (w, k), c in keep.items():
            odf.batch_tune_set(w, k, c)
    info = plan.info()
    assert info["configs"] == expect
    print("plan:", info, flush=True)
    assert info["jobs"] == 40 and sum(info["tiles"]) > 0
    plan.launch()
    torch.cuda.synchronize()
    for j, img in zip(jobs, imgs):
        out, idx = _per_image(j)
        assert torch.equal(j["out"], out) and torch.equal(j["idx"], idx)
        _, _, _, _, O = oracle.filter(img, j["window"], j["kind"], j["p"], j["dist"], j["q"],
                                      aggregates=True)
        check_selection(j["idx"].cpu().numpy(), O)
    plan.close()


def test_batch_graph_replays():
    jobs, _ = _mixed_jobs(24, 2)
    refs = [_per_image(j) for j in jobs]
    plan = odf.BatchPlan(jobs)
    g = plan.capture()
    for rep in range(4):
        for j in jobs:  # eager work between replays: clear the outputs
            j["out"].zero_()
            j["idx"].fill_(255)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for j, (o, i) in zip(jobs, refs):
            assert torch.equal(j["out"], o) and torch.equal(j["idx"], i), rep
    plan.close()


def test_batch_without_idx_and_single_job():
    img = torch.from_numpy(synth.image_corr(77, 91, 0.2, key=4)).to(DEV)
    out = torch.empty_like(img)
    plan = odf.BatchPlan([dict(img=img, out=out, idx=None, window=5, kind=odf.DDF, p=0.25,
                               dist=odf.EXACT)])
    plan.launch()
    ref, _ = odf.filter(img, 5, odf.DDF, 0.25, odf.EXACT)
    assert torch.equal(out, ref)


@pytest.mark.parametrize("window,kind", [(3, 0), (3, 1), (5, 0), (5, 1), (7, 0), (7, 1), (9, 0), (9, 1)])
def test_tile_shapes_give_identical_results(window, kind):
    img = torch.from_numpy(synth.image_corr(150, 170, 0.2, key=window + kind)).to(DEV)
    default = odf.tune_get(window, kind, odf.EXACT, True)
    ref = odf.filter(img, window, kind, 0.25, odf.EXACT)
    tried = 0
    for cfg in range(odf.NUM_TILE_CONFIGS):
        try:
            odf.tune_set(window, kind, odf.EXACT, True, cfg)
        except odf.ODFError:
            continue  # shape not offered for this class
        tried += 1
        o, i = odf.filter(img, window, kind, 0.25, odf.EXACT)
        assert torch.equal(o, ref[0]) and torch.equal(i, ref[1]), cfg
    odf.tune_set(window, kind, odf.EXACT, True, default)
    assert tried >= (1 if (window, kind) == (9, 1) else 2)  # 9x9 DDF: shape 2 only


def test_autotune_picks_a_valid_shape(tmp_path):
    cache = str(tmp_path / "tune.jsonl")
    best, times = odf.autotune(3, odf.DDF, odf.EXACT, True, 512, 512, 3, cache)
    print("autotune 3x3 DDF:", best, times)
    assert len(times) == odf.NUM_TILE_CONFIGS and times[odf.STRIP] > 0  # the strip form is timed
    assert 0 <= best < odf.NUM_TILE_CONFIGS and times[best] == min(t for t in times if t > 0)
    best5, times5 = odf.autotune(5, odf.DDF, odf.EXACT, True, 256, 256, 2, cache)
    assert all(t > 0 for t in times5) and times5[best5] == min(times5)
    odf.tune_set(3, odf.DDF, odf.EXACT, True, 0)
    assert odf.tune_load(cache) == 2
    assert odf.tune_get(3, odf.DDF, odf.EXACT, True) == best


def test_autotune_batch_drives_the_plan(tmp_path):
    """The batch autotuner times the four shapes of a group on its mixed work
    list, sets the fastest in the batch table, which the next plan uses; the
    cache line restores it."""
    cache = str(tmp_path / "tune.jsonl")
    keep = {(w, k): odf.batch_tune_get(w, k) for w in (3, 5, 7, 9) for k in (0, 1)}
    try:
        best, times = odf.autotune_batch(5, odf.BVDF, 2, cache)
        print("autotune_batch 5x5 BVDF:", best, times, flush=True)
        assert len(times) == odf.NUM_TILE_CONFIGS
        assert 0 <= best < odf.NUM_TILE_CONFIGS and all(t > 0 for t in times)
        assert times[best] == min(times)
        jobs, _ = _mixed_jobs(6, 3)
        for j in jobs:
            j["window"], j["kind"] = 5, odf.BVDF
        plan = odf.BatchPlan(jobs)
        assert plan.info()["configs"][2] == best
        plan.launch()
        torch.cuda.synchronize()
        for j in jobs:
            out, idx = _per_image(j)
            assert torch.equal(j["out"], out) and torch.equal(j["idx"], idx)
        plan.close()
        odf.batch_tune_set(5, odf.BVDF, (best + 1) % odf.NUM_TILE_CONFIGS)
        assert odf.tune_load(cache) == 1 and odf.batch_tune_get(5, odf.BVDF) == best
    finally:
        for (w, k), c in keep.items():
            odf.batch_tune_set(w, k, c)


def test_autotune_batch_on_the_callers_jobs():
    """odf_autotune_batch_jobs times each group's shapes on the given jobs and
    sets the table for the groups present; the plan made next uses them and
    still gives the per-image results."""
    keep = {(w, k): odf.batch_tune_get(w, k) for w in (3, 5, 7, 9) for k in (0, 1)}
    try:
        jobs, _ = _mixed_jobs(30, 5)
        res = odf.autotune_batch_jobs(jobs, 2)
        print("autotune_batch_jobs:", res, flush=True)
        present = {"w%d_%s" % (j["window"], ("bvdf", "ddf")[j["kind"]]) for j in jobs}
        assert set(res) == present
        plan = odf.BatchPlan(jobs)
        info = plan.info()
        for g, (best, ms) in res.items():
            # -1: a config the group does not offer (7x7: the 1024-thread shapes)
            timed = [m for m in ms if m >= 0]
            assert len(ms) == odf.NUM_TILE_CONFIGS and ms[best] == min(timed)
            assert (ms[0] < 0 and ms[1] < 0) == (g.startswith("w7") or g.startswith("w9"))
            assert info["ext_tiles"][g] == odf.tile_config(best)
        plan.launch()
        torch.cuda.synchronize()
        for j in jobs:
            out, idx = _per_image(j)
            assert torch.equal(j["out"], out) and torch.equal(j["idx"], idx)
        plan.close()
    finally:
        for (w, k), c in keep.items():
            odf.batch_tune_set(w, k, c)



def test_autotune_batch_7x7_group():
    """The 7x7 groups: the batch autotuner times the shapes they offer (2, 3 and
    the strips; -1 for the 1024-thread shapes) and the plan runs on the fastest,
    bitwise equal to the per-image filter."""
    keep = {(7, k): odf.batch_tune_get(7, k) for k in (0, 1)}
    try:
        best, times = odf.autotune_batch(7, odf.DDF, 1)
        print("autotune_batch 7x7 DDF:", best, times, flush=True)
        assert times[0] < 0 and times[1] < 0 and all(t > 0 for t in times[2:])
        assert best >= 2 and times[best] == min(times[2:])
        jobs, _ = _mixed_jobs(8, 7)
        for j in jobs:
            j["window"], j["kind"] = 7, odf.DDF
        plan = odf.BatchPlan(jobs)
        assert plan.info()["configs"][5] == best
        plan.launch()
        torch.cuda.synchronize()
        for j in jobs:
            out, idx = _per_image(j)
            assert torch.equal(j["out"], out) and torch.equal(j["idx"], idx)
        plan.close()
    finally:
        for (w, k), c in keep.items():
            odf.batch_tune_set(w, k, c)
