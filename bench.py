"""Throughput benchmark of the directional filters on one MI355X.

Default workload (one step): DDF 3x3 on one 1024 x 1024 uint8 RGB image
(smooth synthetic field + 20 edges, correlated impulsive noise 0.20), for
p in {0.25, 0.5} and each pair term {exact angle, minimax q=4, chromaticity}
-- six forward filters per step, timed four ways (a loop of six launches; the
six launches spread over three streams; the six as one planned batch recorded
in a graph, persistent or direct work list) and reported for the fastest.  ``value`` is pixels filtered per second
over the whole step (Mpixels/s).

Also reported on the same JSON line:
  * per-variant kernel throughput (HIP events on the launch stream);
  * ``roofline`` for the dominant kernel against the VALU issue rate;
  * ``forms``: other shapes of the hot path timed the same way;
  * ``cpu_baseline``: the FP64 oracle timed on a bounded pixel sample of the
    same image on the host cores, and the index mismatch rate of the GPU on
    that sample (every mismatch checked to be a near-tie); under
    ``forms_mismatch`` the same for seeded samples of the large-frame forms
    (1 M pixels per 5x5 form, 100 000 per 3x3 and 7x7 form) and of the
    256-image batch (1 M pixels).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-forms] [--no-cpu]
                       [--step-forms loop,streams,persistent,direct] [--copy-probe-mib MiB]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# ------------------------------------------------------------------ cost model
# VALU issue slots per pixel (one slot = one lane-instruction of a binary32
# add/mul/fma/min/max/compare/select).  A transcendental (rsq, sqrt, log)
# counts 2 slots: measured on MI355X with the valu_rates microbenchmark, a
# dependent transcendental + fma chain runs at 1/2.7 of the fma rate.  These
# are the algorithm's operations per output pixel with every unordered pixel
# pair evaluated once; halo recomputation, addressing and LDS traffic are not
# counted.
TRANS = 2
PAIR_SLOTS = {
    "exact": 35 + TRANS,     # dot 3, cross 9, |cross|^2 3, (a.b)^2 1, P*Q, max, rsq, min, r,
                             # r^2, 9-term Horner + 1, quadrant fix-up 3
    "minimax": 38 + TRANS,   # dot 3, cross 9, |cross|^2 3, z 2, exact branch test 6, X 2,
                             # tau 3, two q=4 Horners 8, select, clamp
    "rgb": 14 + TRANS,       # numerators 9, sum of squares 3, sqrt, 2 mul (DDF: +1 fma)
}
L2_SLOTS = 6 + TRANS         # 3 sub, 3 fma/mul, sqrt
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock = 39.3e12 lane-slots/s

# ------------------------------------------------------------------ HBM traffic
# Bytes the DDF 3x3 uint8 forward kernels move to and from HBM on the
# 1024 x 1024 image: rocprofv3 --pmc FETCH_SIZE and --pmc WRITE_SIZE (KiB per
# dispatch, one pass each, from `bench.py --steps 3 --warmup 1 --no-forms
# --no-cpu --step-forms loop,direct --copy-probe-mib 256`), keyed by pair term
# and extended tile for the per-image kernel, and ("batch6", 32, 32) for the
# batch group kernel running the step's six variants in one launch.  Each
# counter is scaled by what it reads for the 256 MiB float32 copy of the same
# run (262144 KiB read, 262144 KiB written): FETCH_SIZE read 131082.2 KiB
# (x 1.99984), WRITE_SIZE 262144.0 KiB (x 1.0).  The figures hold for the
# kernel sources hashed in TRAFFIC_SRC_SHA256; for any other sources bench.py
# reports traffic as null.
TRAFFIC_FETCH_SCALE = 262144.0 / 131082.2
TRAFFIC_WRITE_SCALE = 262144.0 / 262144.0
TRAFFIC_KIB = {  # (dist, ext_w, ext_h): (FETCH_SIZE KiB, WRITE_SIZE KiB)
    ("exact", 32, 32): (4072.6, 6144.0), ("exact", 64, 16): (2895.5, 5056.0),
    ("exact", 32, 16): (4366.9, 6144.0), ("exact", 64, 8): (3186.6, 5056.0),
    ("minimax", 32, 32): (4090.3, 6144.0), ("minimax", 64, 16): (2904.5, 5056.0),
    ("minimax", 32, 16): (4377.9, 6144.0), ("minimax", 64, 8): (3197.0, 5056.0),
    ("rgb", 32, 32): (4072.2, 6144.0), ("rgb", 64, 16): (2892.5, 5056.0),
    ("rgb", 32, 16): (4363.9, 6144.0), ("rgb", 64, 8): (3184.0, 5056.0),
    ("batch6", 32, 32): (21903.4, 36887.7),
}
TRAFFIC_SOURCES = ("fwd.hip", "fwd_launch.h", "batch.hip", "fwd_tile.h", "aggregates.h",
                   "pair_terms.h", "atan_poly.h", "odf_internal.h")
TRAFFIC_SRC_SHA256 = "06c54a4fcc805970c87de27832fb057c33ca7e1eeda85b45d81117963908f226"


def forward_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1009_0958_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_bytes(dist, ext_tile):
    """Calibrated HBM bytes per launch on the 1024 x 1024 image (one filter, or
    for "batch6" the group kernel running all six variants), or None when the
    kernel sources differ from the ones the counters were taken on."""
    key = (dist, int(ext_tile[0]), int(ext_tile[1]))
    if forward_sources_sha256() != TRAFFIC_SRC_SHA256 or key not in TRAFFIC_KIB:
        return None
    fetch, write = TRAFFIC_KIB[key]
    return {"fetch": round(fetch * 1024 * TRAFFIC_FETCH_SCALE),
            "write": round(write * 1024 * TRAFFIC_WRITE_SCALE)}


def slots_per_pixel(window, kind, p, dist):
    h = window // 2
    n = window * window
    pairs = 2 * h * (4 * h + 1) + 2 * h  # unique unordered pairs per pixel: 12 or 40
    box = window * (window - 1) * (3 * window - 1)  # separable box-sum adds per plane
    s = pairs * PAIR_SLOTS[dist] + box + 2 * (n - 1) + 10  # + argmin + prep
    if dist == "rgb" and kind in ("ddf", "acw"):
        s += pairs
    if kind == "acw":
        # DDF aggregates and the eq. (3) product, three centre-weighted
        # objectives per member (2 fma + 1 mul each), and per output pixel the
        # three (pair term x L2) products of the switching statistic
        s += pairs * L2_SLOTS + box + n + 9 * n + 3 * (PAIR_SLOTS[dist] + L2_SLOTS + 2)
    elif kind == "ddf":
        s += pairs * L2_SLOTS + box
        if p == 0.5:
            s += n  # A*D orders like A^(1/2) D^(1/2)
        elif p == 0.25:
            s += 3 * n  # A^3 D orders like A^(3/4) D^(1/4)
        elif p not in (0.0, 1.0):
            s += n * (2 * TRANS + 2)  # (1-p) log2 A + p log2 D per member
    return s


def softmin_slots_per_pixel(window, bwd):
    """VALU lane-slots per output pixel of the softmin relaxation (exact angle,
    DDF with the objective's logarithms).  Forward: the DDF forward's pair terms
    and box sums, per member (1-p) log2 A + p log2 D (2 transcendentals + 2),
    the weight exp2 (1 transcendental + 2) and the weighted sum of colours (3
    fma + 1 add).  Backward: the forward again, per member the weight and
    objective derivatives (8), then per unordered pair the angle gradient (two
    cross products 18, norms and reciprocal 8 + a transcendental, 6 scaling)
    and the L2 gradient (3 sub, reciprocal square root, 3 mul), each
    accumulated into both pixels (12), and the transposed box sums of the
    member gradients (one more set of box sums per plane)."""
    h = window // 2
    n = window * window
    pairs = 2 * h * (4 * h + 1) + 2 * h
    box = window * (window - 1) * (3 * window - 1)
    fwd = (pairs * (PAIR_SLOTS["exact"] + L2_SLOTS) + 2 * box + 10
           + n * (2 * TRANS + 2) + n * (TRANS + 2) + 4 * n)
    if not bwd:
        return fwd
    return (fwd + 8 * n + pairs * (32 + TRANS + 3 + TRANS + 3 + 12) + 2 * box)


# ------------------------------------------------------------------ helpers

def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_launches(torch, fn, reps, warm=3):
    for _ in range(warm):
        fn()
    s, e = _events(torch)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps  # ms per launch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--step-forms", default="loop,streams,persistent,direct",
                    help="step forms to time (comma list of loop, streams, persistent, direct)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one elementwise copy (float32 negation) of this many MiB, "
                         "untimed: the reference kernel for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU hot path "
              "(see the multi-GPU design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    forms_wanted = [f for f in args.step_forms.split(",") if f]
    if not forms_wanted or any(f not in ("loop", "streams", "persistent", "direct")
                               for f in forms_wanted):
        ap.error("--step-forms takes a comma list of loop, streams, persistent, direct")

    import torch
    from paper_1009_0958_amd import odf, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    M = N = 1024
    img_np = synth.image_corr(M, N, 0.20)
    x = torch.from_numpy(img_np).to(dev)
    variants = [(p, d) for p in (0.25, 0.5) for d in ("exact", "minimax", "rgb")]
    DIST = {"exact": odf.EXACT, "minimax": odf.MINIMAX, "rgb": odf.RGB}
    # tile shapes for this image size, chosen by the library's autotuner (untimed)
    tuned = {}
    for d in ("exact", "minimax", "rgb"):
        best, times = odf.autotune(3, odf.DDF, DIST[d], True, M, N, 10)
        tuned["ddf3_%s" % d] = {"config": best, "ext_tile": odf.tile_config(best),
                                "ms_per_shape": [round(t, 5) for t in times]}
    outs = {v: (torch.empty_like(x), torch.empty((M, N), dtype=torch.uint8, device=dev))
            for v in variants}

    def loop_step():
        for (p, d) in variants:
            o, i = outs[(p, d)]
            odf.filter(x, 3, odf.DDF, p, DIST[d], 4, out=o, idx=i)

    # the same six launches spread over three side streams (default priority)
    # joined back into the current stream, so that one launch's last,
    # partially filled wave of workgroups overlaps the next launch
    side = [torch.cuda.Stream(device=dev) for _ in range(3)]

    def streams_step():
        cur = torch.cuda.current_stream(dev)
        fork = cur.record_event()
        for k, (p, d) in enumerate(variants):
            st = side[k % len(side)]
            st.wait_event(fork)
            with torch.cuda.stream(st):
                o, i = outs[(p, d)]
                odf.filter(x, 3, odf.DDF, p, DIST[d], 4, out=o, idx=i)
        for st in side:
            cur.wait_stream(st)

    # the six filters of a step as one planned batch launch, recorded in a
    # graph (classes run concurrently on the plan's streams)
    graphs = {}
    for mode in [f for f in ("persistent", "direct") if f in forms_wanted]:
        plan = odf.BatchPlan([dict(img=x, out=outs[(p, d)][0], idx=outs[(p, d)][1], window=3,
                                   kind=odf.DDF, p=p, dist=DIST[d], q=4) for (p, d) in variants],
                             direct=(mode == "direct"))
        graphs[mode] = (plan, plan.capture())

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        s_, e_ = _events(torch)
        t0_ = time.perf_counter()
        s_.record()
        for _ in range(args.steps):
            fn()
        e_.record()
        torch.cuda.synchronize()
        return s_.elapsed_time(e_) / args.steps, time.perf_counter() - t0_

    step_forms = {"loop_of_launches": timed(loop_step)} if "loop" in forms_wanted else {}
    if "streams" in forms_wanted:
        step_forms["launches_on_3_streams"] = timed(streams_step)
    for mode, (plan, g) in graphs.items():
        step_forms["graph_batch_" + mode] = timed(g.replay)
    best = min(step_forms, key=lambda k: step_forms[k][0])
    ms_step, wall = step_forms[best]
    px_step = len(variants) * M * N
    value = px_step / (ms_step * 1e3)
    # the step's outputs are the filter's: check every form's six outputs against
    # plain launches
    refs = {v: odf.filter(x, 3, odf.DDF, v[0], DIST[v[1]], 4) for v in variants}

    def outputs_match():
        return all(torch.equal(refs[v][0], outs[v][0]) and torch.equal(refs[v][1], outs[v][1])
                   for v in variants)

    step_ok = True
    checked = ([loop_step] if "loop" in forms_wanted else []) + \
        ([streams_step] if "streams" in forms_wanted else [])
    for fn in checked + [g.replay for (_, g) in graphs.values()]:
        for o, i in outs.values():
            o.zero_()
            i.zero_()
        fn()
        torch.cuda.synchronize()
        step_ok = step_ok and outputs_match()

    # per-variant kernel time (HIP events on the launch stream)
    per_variant = {}
    for (p, d) in variants:
        o, i = outs[(p, d)]
        ms = time_launches(torch, lambda: odf.filter(x, 3, odf.DDF, p, DIST[d], 4, out=o, idx=i),
                           max(20, args.steps))
        slots = slots_per_pixel(3, "ddf", p, d) * M * N
        per_variant["ddf3_p%.2f_%s" % (p, d)] = {
            "ms": round(ms, 5), "mpix_s": round(M * N / (ms * 1e3), 1),
            "valu_frac": round(slots / (ms * 1e-3) / PEAK_SLOTS, 4)}
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    if best == "graph_batch_direct":
        # the step is one kernel (the 3x3 DDF group kernel over the tiles of
        # all six variants): time that launch live with events on its stream
        plan = graphs["direct"][0]
        dms = time_launches(torch, plan.launch, max(20, args.steps))
        slots_px = sum(slots_per_pixel(3, "ddf", p, d) for (p, d) in variants) / len(variants)
        npx = len(variants) * M * N
        dname = "batch_direct_kernel ddf3, six variants in one launch"
        tb = traffic_bytes("batch6", (32, 32))
    else:
        dom = max(per_variant, key=lambda k: per_variant[k]["ms"])
        dp, dd = float(dom.split("_")[1][1:]), dom.split("_")[2]
        dms = per_variant[dom]["ms"]
        slots_px = slots_per_pixel(3, "ddf", dp, dd)
        npx = M * N
        dname = "fwd_kernel " + dom
        tb = traffic_bytes(dd, tuned["ddf3_%s" % dd]["ext_tile"])
    dslots = slots_px * npx
    roofline = {
        "bound": "alu", "kernel": dname, "ms_per_launch": round(dms, 5),
        "achieved": round(dslots / (dms * 1e-3) / 1e12, 3), "peak": round(PEAK_SLOTS / 1e12, 2),
        "unit": "T VALU lane-slots/s", "frac": round(dslots / (dms * 1e-3) / PEAK_SLOTS, 4),
        "slots_per_pixel": round(slots_px, 2), "pixels_per_launch": npx,
        "traffic": None,
        "hbm_bytes_per_pixel": 7, "hbm_frac": round(7 * npx / (dms * 1e-3) / 8e12, 5),
    }
    if tb is not None:
        roofline["traffic"] = tb["fetch"] + tb["write"]
        roofline["traffic_fetch_write"] = [tb["fetch"], tb["write"]]
        roofline["traffic_over_algorithmic"] = round((tb["fetch"] + tb["write"]) / (7 * npx), 3)

    forms = {}
    acw_idx = {}
    # seeded samples of the large-frame and batch outputs, checked against the
    # oracle in the cpu_baseline leg (none when that leg is off)
    samples = None if args.no_cpu else {}
    if not args.no_forms:
        for name, fn in (("large_frames",
                          lambda: large_frame_forms(torch, odf, synth, dev, DIST, samples)),
                         ("acwddf", lambda: acwddf_forms(torch, odf, synth, dev, DIST, x, acw_idx)),
                         ("effectiveness", lambda: effectiveness_forms(torch, odf, synth, dev, DIST)),
                         ("batched", lambda: batched_form(torch, odf, synth, dev, samples)),
                         ("differentiable", lambda: differentiable_forms(torch, odf, synth, dev))):
            try:
                forms.update(fn())
            except Exception as exc:  # keep the main line; report the failure
                forms[name + "_error"] = repr(exc)[:300]
            torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(img_np, outs, variants, args.cpu_seconds, acw_idx, samples)

    line = {
        "metric": "Mpixels/s BVDF/DDF 3x3,5x5 fwd & fwd+bwd at 1 GPU; % roofline; mismatch rate",
        "value": round(value, 1), "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "DDF 3x3 forward, 1024x1024 uint8 RGB, correlated impulsive "
                               "noise 0.20, p in {0.25, 0.5} x {exact, minimax q=4, rgb}; "
                               "timed as the fastest of: six launches on one stream or "
                               "spread over three, one batched graph (persistent or direct "
                               "work list)",
                   "image": [M, N], "launches_per_step": len(variants), "parallelism": "none"},
        "wall_s": round(wall, 3),
        "step_forms_ms": {k: round(v[0], 5) for k, v in step_forms.items()}, "step_form": best,
        "step_outputs_match_plain_launch": step_ok,
        "tuned": tuned, "variants": per_variant, "roofline": roofline, "forms": forms,
        "cpu_baseline": cpu,
        "paper_context": {"ddf3_exact_1024x1024_mpix_s": 0.0368,
                          "hardware": "Pentium D 2.66 GHz, C, gcc 3.4.4 (paper, Section II)"},
    }
    print(json.dumps(line), flush=True)


def sample_windows(torch, x, pix, window):
    """The w x w windows (replicated border) of the flat pixel positions pix of
    the uint8 batch x, gathered on the GPU: (k, w, w, 3) uint8 on the host."""
    B, M, N, _ = x.shape
    h = window // 2
    b, rc = np.divmod(pix, M * N)
    r, c = np.divmod(rc, N)
    off = np.arange(-h, h + 1)
    rr = np.clip(r[:, None] + off[None, :], 0, M - 1)
    cc = np.clip(c[:, None] + off[None, :], 0, N - 1)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(x.device)  # noqa: E731
    return x[t(b[:, None, None]), t(rr[:, :, None]), t(cc[:, None, :])].cpu().numpy()


def mismatch_sample(B, M, N, k, seed):
    """k seeded flat pixel positions of a B x M x N batch (all when k >= BMN)."""
    n = B * M * N
    if k >= n:
        return np.arange(n)
    return np.sort(np.random.default_rng(seed).choice(n, k, replace=False))


def large_frame_forms(torch, odf, synth, dev, DIST, samples=None):
    """7680 x 4320 frame (3x3 BVDF, 5x5 and 7x7) and 64 x 1920 x 1080 frames
    (5x5), correlated noise 0.15 (tile shapes autotuned per class first,
    untimed).  With ``samples`` (a dict), the windows of 1 M seeded pixels
    (5x5; 100 000 for 3x3 and 7x7) and the GPU's index there are kept for the
    oracle check of the cpu_baseline leg."""
    forms = {}
    for w, kk in ((3, odf.BVDF), (5, odf.BVDF), (5, odf.DDF), (7, odf.BVDF), (7, odf.DDF)):
        for d in ("exact", "minimax", "rgb"):
            odf.autotune(w, kk, DIST[d], True, 1024, 1024, 3)
    for tag, shape, key in (("7680x4320", (1, 4320, 7680), 5), ("64x1920x1080", (64, 1080, 1920), 6)):
        B, M, N = shape
        imgs = np.stack([synth.image_corr(M, N, 0.15, key=key * 100 + b) for b in range(B)])
        big = torch.from_numpy(imgs).to(dev)
        del imgs
        bo = torch.empty_like(big)
        bi = torch.empty((B, M, N), dtype=torch.uint8, device=dev)
        npx = B * M * N
        for w, kind, p in ((3, "bvdf", 0.0), (5, "bvdf", 0.0), (5, "ddf", 0.25), (7, "bvdf", 0.0),
                           (7, "ddf", 0.25)):
            if tag != "7680x4320" and w in (3, 7):
                continue
            for d in ("exact", "minimax", "rgb"):
                kk = odf.BVDF if kind == "bvdf" else odf.DDF
                ms = time_launches(torch, lambda: odf.filter(big, w, kk, p, DIST[d], 4, out=bo,
                                                             idx=bi), 5, warm=1)
                name = "%s%d_%s_%s" % (kind, w, d, tag)
                forms[name] = {
                    "mpix_s": round(npx / (ms * 1e3), 1), "ms": round(ms, 3),
                    "valu_frac": round(slots_per_pixel(w, kind, p, d) * npx / (ms * 1e-3)
                                       / PEAK_SLOTS, 4)}
                if samples is not None:
                    key = (tag, w)
                    if key not in samples.setdefault("windows", {}):
                        pix = mismatch_sample(B, M, N, 1_000_000 if w == 5 else 100_000,
                                              7000 + 10 * w + key[0].count("x"))
                        samples["windows"][key] = (pix, sample_windows(torch, big, pix, w))
                    pix = samples["windows"][key][0]
                    gidx = bi.reshape(-1)[torch.from_numpy(pix).to(dev)].cpu().numpy()
                    samples.setdefault("cases", []).append((name, key, w, kind, p, d, gidx))
        del big, bo, bi
    return forms


def acwddf_forms(torch, odf, synth, dev, DIST, x1k, acw_idx):
    """ACWDDF (lambda = 2, T = 10.8) on the 1024 x 1024 image (3x3 and 5x5)
    and on a 7680 x 4320 frame (3x3), each pair term, tuned tile shapes; the
    1024 x 1024 3x3 index maps are kept for the oracle's mismatch count.  Also
    CWVMF^2 and CWDDF^2 (exact) on the 1024 x 1024 image."""
    forms = {}
    big = torch.from_numpy(synth.image_corr(4320, 7680, 0.15, key=500)).to(dev)
    for w in (3, 5):
        for d in ("exact", "minimax", "rgb"):
            best, _ = odf.autotune(w, odf.ACWDDF, DIST[d], True, 1024, 1024, 5)
            cases = [("1024x1024", x1k)] + ([("7680x4320", big)] if w == 3 else [])
            for tag, img in cases:
                M, N = img.shape[:2]
                o = torch.empty_like(img)
                i = torch.empty((M, N), dtype=torch.uint8, device=dev)
                ms = time_launches(torch, lambda: odf.acwddf(img, w, DIST[d], 4, 2, 10.8, out=o,
                                                             idx=i), 10, warm=2)
                forms["acwddf%d_%s_%s" % (w, d, tag)] = {
                    "mpix_s": round(M * N / (ms * 1e3), 1), "ms": round(ms, 4),
                    "ext_tile": odf.tile_config(best),
                    "valu_frac": round(slots_per_pixel(w, "acw", 0.5, d) * M * N / (ms * 1e-3)
                                       / PEAK_SLOTS, 4),
                    "switched_to_ddf": round(float((i != (w * w - 1) // 2).float().mean()), 4)}
                if tag == "1024x1024" and w == 3:
                    acw_idx[d] = i.cpu().numpy()
    # the centre-weighted filters on their own (eq. 9), level k = 2, on the
    # ACWDDF kernels and their tuned tile shapes
    M, N = x1k.shape[:2]
    o = torch.empty_like(x1k)
    i = torch.empty((M, N), dtype=torch.uint8, device=dev)
    for w in (3, 5):
        for name, kind, d in (("cwvmf", odf.CWVMF, "rgb"), ("cwddf", odf.CWDDF, "exact")):
            ms = time_launches(torch, lambda: odf.cw_filter(x1k, w, kind, 2, DIST[d], 4, out=o,
                                                            idx=i), 10, warm=2)
            forms["%s%d_k2_1024x1024" % (name, w)] = {"mpix_s": round(M * N / (ms * 1e3), 1),
                                                      "ms": round(ms, 4)}
    del big
    return forms


def effectiveness_forms(torch, odf, synth, dev, DIST):
    """The paper's effectiveness check on synthetic stand-ins: a clean
    1024 x 1024 image corrupted on the GPU by eq. (8) (phi = 0.10, 0.15,
    channel probabilities 0.25), filtered by BVDF (Experiment 1) and ACWDDF
    (Experiment 2) with each pair term, scored by MAE / PSNR on the GPU; plus
    the noise and quality kernels' rates on a 7680 x 4320 frame."""
    clean = torch.from_numpy(synth.smooth_image(1024, 1024, synth.rng_for(9, 0))).to(dev)
    table = {}
    for phi in (0.10, 0.15):
        noisy = odf.noise_eq8(clean, phi, seed=1009)
        row = {"noisy": noisy}
        for d in ("exact", "minimax", "rgb"):
            row["bvdf_" + d] = odf.filter(noisy, 3, odf.BVDF, 0.0, DIST[d], 4)[0]
            row["acwddf_" + d] = odf.acwddf(noisy, 3, DIST[d], 4, 2, 10.8)[0]
        names = list(row)
        mae, psnr = odf.quality(torch.stack([row[k] for k in names]),
                                clean.unsqueeze(0).expand(len(names), -1, -1, -1).contiguous())
        table["phi%.2f" % phi] = {k: {"mae": round(float(m), 4), "psnr": round(float(p_), 3)}
                                  for k, m, p_ in zip(names, mae.tolist(), psnr.tolist())}
    big = torch.from_numpy(synth.smooth_image(4320, 7680, synth.rng_for(9, 1))).to(dev)
    out = torch.empty_like(big)
    npx = 4320 * 7680
    ms_noise = time_launches(torch, lambda: odf.noise_eq8(big, 0.15, seed=5, out=out), 10, warm=2)
    ws = torch.empty(16, dtype=torch.uint8, device=dev)
    ms_q = time_launches(torch, lambda: odf.quality(out, big, workspace=ws), 10, warm=2)
    rates = {"noise_eq8_7680x4320": {"ms": round(ms_noise, 4), "mpix_s": round(npx / (ms_noise * 1e3), 1),
                                     "hbm_GBps": round(6 * npx / (ms_noise * 1e6), 1)},
             "quality_7680x4320": {"ms": round(ms_q, 4), "mpix_s": round(npx / (ms_q * 1e3), 1),
                                   "hbm_GBps": round(6 * npx / (ms_q * 1e6), 1)}}
    return {"effectiveness_1024x1024_eq8": table, **rates}


def batched_form(torch, odf, synth, dev, samples=None):
    """256 uint8 images of mixed size (64..2048 x 64..1536), window, kind and
    noise: one planned launch captured in a graph (direct and persistent form;
    one kernel per window and kind), against a loop of per-image launches of
    the same jobs (tile shapes from the autotuned table)."""
    specs = synth.mixed_batch_specs(256)
    imgs = synth.mixed_batch_images(specs, workers=16)
    # tile shapes of the per-image launches of the loop (untimed)
    tuned = {}
    for w in (3, 5):
        for kind in (odf.BVDF, odf.DDF):
            best, _ = odf.autotune(w, kind, odf.EXACT, True, 1024, 1024, 5)
            tuned[f"w{w}_{'ddf' if kind else 'bvdf'}"] = odf.tile_config(best)
    jobs = []
    for s_, im in zip(specs, imgs):
        t = torch.from_numpy(im).to(dev)
        jobs.append(dict(img=t, out=torch.empty_like(t),
                         idx=torch.empty(t.shape[:2], dtype=torch.uint8, device=dev),
                         window=s_["window"], kind=s_["kind"], p=s_["p"], dist=odf.EXACT, q=4))
    del imgs
    npx = sum(int(j["img"].shape[0] * j["img"].shape[1]) for j in jobs)
    loop_out = [(torch.empty_like(j["out"]), torch.empty_like(j["idx"])) for j in jobs]

    def loop():
        for j, (o, i) in zip(jobs, loop_out):
            odf.filter(j["img"], j["window"], j["kind"], j["p"], odf.EXACT, 4, out=o, idx=i)

    ms_loop = time_launches(torch, loop, 3, warm=1)

    def same_as_loop():
        return all(torch.equal(j["out"], o) and torch.equal(j["idx"], i)
                   for j, (o, i) in zip(jobs, loop_out))

    res = {}
    for name, direct in (("direct", True), ("persistent", False)):
        for j in jobs:
            j["out"].zero_()
            j["idx"].zero_()
        plan = odf.BatchPlan(jobs, direct=direct)
        graph = plan.capture()
        ms = time_launches(torch, graph.replay, 5, warm=2)
        res[name] = (ms, same_as_loop(), plan.info())
        plan.close()
    if samples is not None:
        # 1 M seeded pixels over the whole batch (the outputs of the last
        # replay of the persistent graph, bitwise equal to the direct one's)
        sizes = np.array([int(j["img"].shape[0] * j["img"].shape[1]) for j in jobs])
        start = np.concatenate([[0], np.cumsum(sizes)])
        flat = mismatch_sample(1, 1, int(start[-1]), 1_000_000, 7100)
        which = np.searchsorted(start, flat, side="right") - 1
        for i in np.unique(which):
            pix = flat[which == i] - start[i]
            j = jobs[i]
            win = sample_windows(torch, j["img"][None], pix, j["window"])
            gidx = j["idx"].reshape(-1)[torch.from_numpy(pix).to(dev)].cpu().numpy()
            samples.setdefault("batch", []).append((j["window"], j["kind"], j["p"], win, gidx))
    ms_direct, same_d, info = res["direct"]
    ms_pers, same_p, _ = res["persistent"]
    return {"batched_256_mixed": {
        "mpix": round(npx / 1e6, 2), "loop_tile_shapes": tuned,
        "batch_tile_shapes": {"w3_ddf": [32, 32], "other": [32, 16]},
        "direct_graph_ms": round(ms_direct, 3), "direct_graph_mpix_s": round(npx / (ms_direct * 1e3), 1),
        "persistent_graph_ms": round(ms_pers, 3),
        "persistent_graph_mpix_s": round(npx / (ms_pers * 1e3), 1),
        "loop_ms": round(ms_loop, 3),
        "loop_mpix_s": round(npx / (ms_loop * 1e3), 1),
        "speedup_direct_vs_loop": round(ms_loop / ms_direct, 3),
        "bitwise_equal_to_loop": bool(same_d and same_p), "tiles_per_class": info["tiles"]}}


def plain_softmin(torch, x, w, p, tau):
    """Unfused PyTorch form of the DDF softmin relaxation (every window's n^2
    pair terms materialised, autograd backward): the plain form the HIP kernels
    are compared with."""
    F = torch.nn.functional
    B, M, N, _ = x.shape
    h, n = w // 2, w * w
    xp = F.pad(x.permute(0, 3, 1, 2), (h, h, h, h), mode="replicate")
    win = xp.unfold(2, w, 1).unfold(3, w, 1).reshape(B, 3, M, N, n).permute(0, 2, 3, 4, 1)
    zero = (win == 0).all(-1, keepdim=True)
    d = torch.where(zero, torch.ones_like(win), win)
    a, b = d.unsqueeze(-2), d.unsqueeze(-3)
    dot = (a * b).sum(-1)
    c0 = a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1]
    c1 = a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2]
    c2 = a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]
    th = torch.atan2(torch.sqrt(c0 * c0 + c1 * c1 + c2 * c2 + 1e-30), dot)
    A = th.sum(-1)
    D = torch.sqrt(((win.unsqueeze(-2) - win.unsqueeze(-3)) ** 2).sum(-1) + 1e-30).sum(-1)
    om = A.pow(1 - p) * D.pow(p)
    pi = torch.softmax(-om / tau, dim=-1)
    return (pi.unsqueeze(-1) * win).sum(-2)


def differentiable_forms(torch, odf, synth, dev):
    """16 x 512 x 512 float32, DDF 5x5 p = 0.25: hard fwd + one-hot bwd, and
    softmin fwd + bwd at tau 0.01 and 0.1; a plain PyTorch softmin on 2 of the
    images for comparison."""
    forms = {}
    x = torch.from_numpy(synth.float_batch(16, 512, 512, 0.1)).to(dev)
    dy = torch.randn_like(x)
    npx = 16 * 512 * 512
    out = torch.empty_like(x)
    idx = torch.empty(x.shape[:3], dtype=torch.uint8, device=dev)
    ms_f = time_launches(torch, lambda: odf.filter(x, 5, odf.DDF, 0.25, odf.EXACT, 4, out=out,
                                                   idx=idx), 10)
    ms_b = time_launches(torch, lambda: odf.backward_hard(idx, dy, 5), 10)
    forms["ddf5_f32_16x512x512_hard"] = {
        "fwd_ms": round(ms_f, 3), "bwd_ms": round(ms_b, 3),
        "fwd_bwd_mpix_s": round(npx / ((ms_f + ms_b) * 1e3), 1),
        "fwd_valu_frac": round(slots_per_pixel(5, "ddf", 0.25, "exact") * npx / (ms_f * 1e-3)
                               / PEAK_SLOTS, 4),
        "bwd_hbm_GBps": round(npx * 25 / (ms_b * 1e-3) / 1e9, 1),
        "bwd_hbm_frac": round(npx * 25 / (ms_b * 1e-3) / 8e12, 4)}
    ws = torch.empty(odf.lib().odf_softmin_bwd_workspace(16, 512, 512, 5, odf.DDF),
                     dtype=torch.uint8, device=dev)
    for tau in (0.01, 0.1):
        ms_sf = time_launches(torch, lambda: odf.softmin_forward(x, 5, odf.DDF, 0.25, tau), 5)
        ms_sb = time_launches(torch, lambda: odf.softmin_backward(x, dy, 5, odf.DDF, 0.25, tau,
                                                                  workspace=ws), 5)
        forms["ddf5_f32_16x512x512_softmin_tau%g" % tau] = {
            "fwd_ms": round(ms_sf, 3), "bwd_ms": round(ms_sb, 3),
            "fwd_bwd_mpix_s": round(npx / ((ms_sf + ms_sb) * 1e3), 1),
            "fwd_valu_frac": round(softmin_slots_per_pixel(5, False) * npx / (ms_sf * 1e-3)
                                   / PEAK_SLOTS, 4),
            "bwd_valu_frac": round(softmin_slots_per_pixel(5, True) * npx / (ms_sb * 1e-3)
                                   / PEAK_SLOTS, 4)}
    # plain PyTorch on 2 images (its n^2 intermediates take several GB per image)
    xs = x[:2].clone().requires_grad_(True)
    g = dy[:2].contiguous()

    def plain():
        xs.grad = None
        y = plain_softmin(torch, xs, 5, 0.25, 0.1)
        y.backward(g)

    ms_plain = time_launches(torch, plain, 2, warm=1)
    ref = odf.softmin_backward(x[:2].contiguous(), g, 5, odf.DDF, 0.25, 0.1)
    rel = ((xs.grad - ref).abs().max() / ref.abs().max()).item()
    forms["ddf5_f32_2x512x512_softmin_tau0.1_plain_torch"] = {
        "fwd_bwd_ms": round(ms_plain, 3),
        "fwd_bwd_mpix_s": round(2 * 512 * 512 / (ms_plain * 1e3), 1),
        "max_rel_diff_vs_hip": rel}
    return forms


def acwddf_mismatch(oracle, img_np, acw_idx, codes, k=20000):
    """ACWDDF 3x3 index mismatches against the oracle on k seeded pixels, and
    whether each one is undetermined at binary32 precision (S within 1e-5 of
    T, or a near-tie within 1e-6 between members of different colours in one
    of the four selections)."""
    M, N = img_np.shape[:2]
    pix = np.sort(np.random.default_rng(1010).choice(M * N, k, replace=False))
    rr, cc = pix // N, pix % N
    cols = np.stack([img_np[np.clip(rr + u // 3 - 1, 0, M - 1), np.clip(cc + u % 3 - 1, 0, N - 1)]
                     for u in range(9)], axis=1)
    res = {}
    for d, g_idx in acw_idx.items():
        _, o_idx, S, dg = oracle.acwddf_at(img_np, pix, 3, codes[d], 4, 2, 10.8)
        g = g_idx.reshape(-1)[pix]
        diff = g != o_idx
        amb = (S != 0) & (np.abs(S - 10.8) <= 1e-5 * 10.8)
        rows = np.arange(k)
        for j in range(4):
            O = dg[:, 9 * j:9 * (j + 1)]
            first = O.argmin(1)
            near = O <= O[rows, first][:, None] * (1 + 1e-6)
            amb |= np.any(near & np.any(cols != cols[rows, first][:, None], axis=2), axis=1)
        res[d] = {"index_mismatch": int(diff.sum()), "index_compared": k,
                  "mismatches_all_undetermined": bool(np.all(amb[diff]))}
    return res


def host_cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def sampled_mismatch(oracle, samples, codes):
    """Index mismatches of the kept samples against the oracle, per form (each
    sampled pixel's window given to the oracle as a w x w patch of its own),
    and whether every mismatch is a near-tie (the oracle's objective of the
    GPU's choice within 1e-6 relative of the minimum)."""
    def check(win, gidx, w, kind, p, d):
        k = win.shape[0]
        centre = np.arange(k) * w * w + (w * w) // 2
        _, _, _, _, O = oracle.filter_at(win, centre, w, kind, p, codes[d])
        g = gidx.astype(np.int64)
        first = O.argmin(1)
        diff = g != first
        og = O[np.arange(k), g]
        near = (og <= O.min(1) * (1 + 1e-6)) | ((O.min(1) == 0) & (og == 0))
        return int(diff.sum()), k, bool(np.all(near[diff]))

    res = {}
    t0 = time.perf_counter()
    for name, key, w, kind, p, d, gidx in samples.get("cases", []):
        win = samples["windows"][key][1]
        m, k, ok = check(win, gidx, w, oracle.DDF if kind == "ddf" else oracle.BVDF, p, d)
        res[name] = {"index_mismatch": m, "index_compared": k, "mismatches_all_near_ties": ok}
    if samples.get("batch"):
        m = k = 0
        ok = True
        for w, kind, p, win, gidx in samples["batch"]:
            mi, ki, oki = check(win, gidx, w, kind, p, "exact")
            m, k, ok = m + mi, k + ki, ok and oki
        res["batched_256_mixed"] = {"index_mismatch": m, "index_compared": k,
                                    "mismatches_all_near_ties": ok}
    res["seconds"] = round(time.perf_counter() - t0, 1)
    return res


def cpu_baseline(img_np, outs, variants, seconds, acw_idx=None, samples=None):
    """FP64 oracle on a seeded pixel sample of the same image, all host threads;
    also the index mismatch rate of the kept samples of the other forms."""
    import oracle

    M, N = img_np.shape[:2]
    codes = {"exact": 0, "minimax": 1, "rgb": 2}
    rng = np.random.default_rng(1009)
    # calibrate on 200000 pixels per variant, then size the work to ~seconds:
    # a seeded pixel sample, or whole-image passes repeated when one pass is short
    probe = rng.integers(0, M * N, 200000)
    t0 = time.perf_counter()
    for (p, d) in variants:
        oracle.filter_at(img_np, probe, 3, oracle.DDF, p, codes[d])
    per_px = (time.perf_counter() - t0) / (200000 * len(variants))
    want = seconds / (per_px * len(variants))
    k = int(min(M * N, max(4000, want)))
    reps = max(1, int(round(want / (M * N)))) if k == M * N else 1
    pix = np.arange(M * N) if k == M * N else np.sort(rng.choice(M * N, k, replace=False))
    t0 = time.perf_counter()
    mism = 0
    near = True
    for r in range(reps):
        for (p, d) in variants:
            _, o_idx, _, _, O = oracle.filter_at(img_np, pix, 3, oracle.DDF, p, codes[d])
            if r:
                continue
            g = outs[(p, d)][1].cpu().numpy().reshape(-1)[pix].astype(np.int64)
            diff = g != o_idx
            mism += int(diff.sum())
            og = O[np.arange(k), g]
            near &= bool(np.all((og <= O.min(1) * (1 + 1e-6))[diff]))
    dt = time.perf_counter() - t0
    what = ("%d seeded pixels of" % k) if k < M * N else ("%d pass(es) over all pixels of" % reps)
    return {"value": round(reps * k * len(variants) / dt / 1e6, 5), "unit": "Mpixels/s",
            "cores": oracle.threads(), "cpu_model": host_cpu_model(), "kind": "oracle",
            "sample": "%s the 1024x1024 image x %d variants, DDF 3x3 (%.1f s)"
                      % (what, len(variants), dt),
            "index_mismatch": mism, "index_compared": k * len(variants),
            "mismatches_all_near_ties": near,
            "acwddf3_1024x1024": acwddf_mismatch(oracle, img_np, acw_idx, codes) if acw_idx
            else None,
            "forms_mismatch": sampled_mismatch(oracle, samples, codes) if samples else None}


if __name__ == "__main__":
    main()
