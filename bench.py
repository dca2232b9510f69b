"""Throughput benchmark of the directional filters on one MI355X.

Step (the ``value``): DDF 5x5 (p = 1/4, exact angle of eq. 2) on one
7680 x 4320 uint8 RGB frame (smooth synthetic field + 20 edges, correlated
impulsive noise 0.15), one forward launch per step with the tile shape the
library's autotuner picks for that frame (untimed).  ``value`` is pixels
filtered per second (Mpixels/s), the mean over the timed steps between HIP
events on the launch stream (after --prewarm-ms of untimed steps and the W
warm-up steps).

Also reported on the same JSON line:
  * ``roofline`` for the step's kernel (the only kernel of the step) against
    the VALU issue rate, from the same events;
  * ``forms``: the other shapes of the hot path, each timed the same way
    (DDF 3x3 six variants on a 1024 x 1024 image as launches, streams and a
    batched graph; 7680 x 4320 and 64 x 1920 x 1080 frames at 3x3 / 5x5 / 7x7;
    ACWDDF and the centre-weighted filters; eq. 8 noise and MAE / PSNR; the
    256-image mixed batch; hard and softmin fwd+bwd on 16 x 512 x 512 float32);
  * ``cpu_baseline``: the FP64 oracle on a band of whole rows of the step's
    frame (about --cpu-seconds of work) on the host cores, the GPU's index
    mismatches on that band (each checked to be a near-tie, and split by
    whether the two members are collinear colours and whether the oracle's
    objectives tie exactly), and under ``forms_mismatch`` the same for the
    six DDF 3x3 variants over the whole 1024 x 1024 image and seeded samples of
    the large-frame forms (1 M pixels per 5x5 form, 100 000 per 3x3 and 7x7
    form) and of the 256-image batch (1 M pixels).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--prewarm-ms MS] [--no-forms] [--no-cpu]
                       [--forms six_variants,large_frames,acwddf,effectiveness,batched,
                        differentiable] [--step-forms loop,streams,direct]
                       [--copy-probe-mib MiB]
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
# VALU issue slots per pixel (one slot = one lane-instruction of a binary32 or
# binary64 add/mul/fma/min/max/compare/select/convert).  A transcendental (rsq,
# sqrt, log, exp) counts 2 slots: measured on MI355X with the valu_rates
# microbenchmark, a dependent transcendental + fma chain runs at 1/2.7 of the
# fma rate.  These are the operations per output pixel of the arithmetic that
# runs, with every unordered pixel pair evaluated once and a member's own
# conversions hoisted out of its pair loop; halo recomputation, addressing and
# LDS traffic are not counted.  uint8 pixels carry exact integer products (the
# cross product's squared norm is Lagrange's identity in binary64), float32
# pixels form their cross products and chromaticity numerators in binary64.
TRANS = 2
PAIR_SLOTS = {
    # dot 3, (a.b)^2 1, Lagrange |a|^2|b|^2 - (a.b)^2 in binary64 with its
    # conversions 5, min 1, P*Q 1, rsq, clamp 1, r 1, r^2 1, 9 Horner fma,
    # r*poly 1, quadrant fix-up 3
    ("exact", True): 27 + TRANS,
    # dot 3, z 2, branch test z < 1/2 and |z - 1/2| <= 2^-20 3, Lagrange 5,
    # X = |a|^2|b|^2 (1 + z) 3, P*X 1, rsq, clamp 1, tau 1, two q = 4 Horners 8,
    # clamp at 0 1, select 1
    ("minimax", True): 29 + TRANS,
    # three integer numerators (mul + fma) 6, sum of squares 3, sqrt, 2 mul
    ("rgb", True): 11 + TRANS,
    # dot 3, (a.b)^2 1, binary64 cross product: 3 conversions, 3 mul, 3 fma,
    # squared norm 3 + conversion 1, min 1, P*Q 1, floor at the smallest
    # normal 1, rsq, r 1, r^2 1, 9 Horner fma, r*poly 1, quadrant fix-up 3,
    # sign of a.b fix-up 3
    ("exact", False): 38 + TRANS,
    # dot 3, z 2, branch test 3, binary64 cross product 13, X 3, P*X 1,
    # floor 1, rsq, tau 1, two Horners 8, clamp 1, select 1
    ("minimax", False): 37 + TRANS,
    # binary64 channel sum of b 2 (+ 3 conversions), numerators 3 x (2 mul +
    # sub) 9, conversions 3, sum of squares 3, sqrt, 2 mul
    ("rgb", False): 22 + TRANS,
}
L2_SLOTS = {
    # uint8 exact / minimax: |a - b|^2 = |a|^2 + |b|^2 - 2 a.b from the angle's
    # dot product (add, fma), the zero-pixel test 1, sqrt
    ("exact", True): 3 + TRANS, ("minimax", True): 3 + TRANS,
    # otherwise: 3 sub, sum of squares 3 (+ the uint8 zero-pixel test), sqrt
    ("rgb", True): 7 + TRANS,
    ("exact", False): 6 + TRANS, ("minimax", False): 6 + TRANS, ("rgb", False): 6 + TRANS,
}
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock = 39.3e12 lane-slots/s

# ------------------------------------------------------------------ HBM traffic
# Bytes the step's kernel (DDF 5x5 exact, uint8, strip form of 32 x 16 bands,
# on the 7680 x 4320 frame) and the six-variant DDF 3x3 batch kernel (32 x 16
# tiles, on the 1024 x 1024 image) move to and from HBM: rocprofv3 --pmc
# FETCH_SIZE and --pmc WRITE_SIZE (KiB per dispatch, one pass each, from
# `bench.py --steps 3 --warmup 1 --no-cpu --forms
# six_variants,large_frames,batched,differentiable --step-forms loop,direct
# --copy-probe-mib 256 --tune-cache <file>`), keyed by form and extended tile
# (or band).  Each counter is scaled by what it reads for the 256 MiB float32
# copy of the same run (262144 KiB read, 262144 KiB written): FETCH_SIZE read
# 131085.5 KiB (x 1.99979), WRITE_SIZE 262144.0 KiB (x 1.0).  The figures hold
# for the kernel code hashed in TRAFFIC_SRC_SHA256 (comments and indentation
# excluded); for any
# other code bench.py reports traffic as null.
TRAFFIC_FETCH_SCALE = 262144.0 / 131085.5
TRAFFIC_WRITE_SCALE = 262144.0 / 262144.0
TRAFFIC_KIB = {  # (form, ext_w, ext_h): (FETCH_SIZE KiB, WRITE_SIZE KiB)
    ("ddf5_exact_7680x4320_strip", 32, 16): (51784.7, 129657.9),
    ("batch6", 32, 16): (21001.6, 36888.0),
}
TRAFFIC_SOURCES = ("fwd.hip", "fwd5.hip", "fwd5s.hip", "fwd_launch.h", "fwd_strip.h", "batch.hip",
                   "fwd_tile.h", "aggregates.h", "pair_terms.h", "canon.h", "atan_poly.h",
                   "odf_internal.h")
TRAFFIC_SRC_SHA256 = "321fb4117fa9493761d1644d027873b17247d3c30bd0b81522068f963120b72f"


def forward_sources_sha256():
    """SHA-256 of the forward kernels' sources with their // comments, the
    blanks around each line and empty lines removed: a change of code changes
    it, a change of comments or indentation does not."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1009_0958_amd", "csrc", name)) as f:
            for line in f:
                code = re.sub(r"//.*", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def traffic_bytes(dist, ext_tile):
    """Calibrated HBM bytes per launch of the step's kernel ("ddf5_exact_7680x4320",
    "..._strip" for the strip form) or of the six-variant batch kernel ("batch6"),
    for the extended tile (or band) it ran on, or None when no counters were
    taken for it or the kernel sources differ from the ones they were taken on."""
    key = (dist, int(ext_tile[0]), int(ext_tile[1]))
    if forward_sources_sha256() != TRAFFIC_SRC_SHA256 or key not in TRAFFIC_KIB:
        return None
    fetch, write = TRAFFIC_KIB[key]
    return {"fetch": round(fetch * 1024 * TRAFFIC_FETCH_SCALE),
            "write": round(write * 1024 * TRAFFIC_WRITE_SCALE)}


def slots_per_pixel(window, kind, p, dist, u8=True):
    h = window // 2
    n = window * window
    pairs = 2 * h * (4 * h + 1) + 2 * h  # unique unordered pairs per pixel: 12, 40 or 84
    box = window * (window - 1) * (3 * window - 1)  # separable box-sum adds per plane
    s = pairs * PAIR_SLOTS[(dist, u8)] + box + 2 * (n - 1) + 10  # + argmin + prep
    l2 = L2_SLOTS[(dist, u8)]
    if dist == "rgb" and kind in ("ddf", "acw"):
        s += pairs  # eq. (10) fma
    if kind == "acw":
        # DDF aggregates and the eq. (3) product, three centre-weighted
        # objectives per member (2 fma + 1 mul each), and per output pixel the
        # three (pair term x L2) products of the switching statistic
        s += pairs * l2 + box + n + 9 * n + 3 * (PAIR_SLOTS[(dist, u8)] + l2 + 2)
    elif kind == "ddf":
        s += pairs * l2 + box
        if p == 0.5:
            s += n  # A*D orders like A^(1/2) D^(1/2)
        elif p == 0.25:
            s += 3 * n  # A^3 D orders like A^(3/4) D^(1/4)
        elif p not in (0.0, 1.0):
            s += n * (2 * TRANS + 2)  # (1-p) log2 A + p log2 D per member
    return s


def softmin_slots_per_pixel(window, bwd):
    """VALU lane-slots per output pixel of the softmin relaxation (float32
    pixels, exact angle, DDF with the objective's logarithms).  Forward: the
    DDF forward's pair terms and box sums, per member (1-p) log2 A + p log2 D
    (2 transcendentals + 2), the weight exp2 (1 transcendental + 2) and the
    weighted sum of colours (3 fma + 1 add).  Backward: the forward again, per
    member the weight and objective derivatives (8), then per unordered pair the
    angle gradient (two cross products 18, norms and reciprocal 8 + a
    transcendental, 6 scaling) and the L2 gradient (3 sub, reciprocal square
    root, 3 mul), each accumulated into both pixels (12), and the transposed box
    sums of the member gradients (one more set of box sums per plane)."""
    h = window // 2
    n = window * window
    pairs = 2 * h * (4 * h + 1) + 2 * h
    box = window * (window - 1) * (3 * window - 1)
    fwd = (pairs * (PAIR_SLOTS[("exact", False)] + L2_SLOTS[("exact", False)]) + 2 * box + 10
           + n * (2 * TRANS + 2) + n * (TRANS + 2) + 4 * n)
    if not bwd:
        return fwd
    return (fwd + 8 * n + pairs * (32 + TRANS + 3 + TRANS + 3 + 12) + 2 * box)


# ------------------------------------------------------------------ helpers

def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def time_launches(torch, fn, reps, warm=3):
    """Mean ms per call of fn over reps calls (after warm untimed calls),
    between HIP events on torch's current stream."""
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


TUNE_CACHE = None  # set by --tune-cache
TUNE_CACHED = False  # the cache existed when the run started: replay it, tune nothing
TUNE_REPLAY = []  # the cache's per-image entries in the order the first run tuned them


def autotune(odf, window, kind, dist, u8, M, N, reps):
    """The library's autotuner, or, when --tune-cache named an existing file at
    start-up, the next entry of that cache for this class: a class tuned twice
    (on different sizes) gets the same config at each point of the run as in
    the run that wrote the cache.  Returns (config, ms per config or [])."""
    if TUNE_CACHED:
        for n, e in enumerate(TUNE_REPLAY):
            if e[:4] == (window, kind, dist, int(bool(u8))):
                del TUNE_REPLAY[n]
                odf.tune_set(window, kind, dist, u8, e[4])
                return e[4], []
        return odf.tune_get(window, kind, dist, u8), []
    return odf.autotune(window, kind, dist, u8, M, N, reps, cache_path=TUNE_CACHE)


def tune_batch(odf, jobs, tag):
    """The batch groups' tile shapes for these jobs: loaded from the cache
    file --tune-cache + "." + tag when it exists, else tuned on the jobs
    (untimed; written there when --tune-cache is given).  Returns {group:
    {config, ext_tile, ms_per_config}} for the groups the jobs use."""
    path = TUNE_CACHE + "." + tag if TUNE_CACHE else None
    if TUNE_CACHED and path and os.path.exists(path) and os.path.getsize(path) > 0:
        odf.tune_load(path)
        groups = {f"w{j['window']}_{'ddf' if j['kind'] else 'bvdf'}" for j in jobs}
        res = {g: (odf.batch_tune_get(int(g[1]), int(g.endswith("ddf"))), []) for g in groups}
    else:
        res = odf.autotune_batch_jobs(jobs, 2, path)
    return {g: {"config": b, "ext_tile": odf.tile_config(b),
                "ms_per_config": [round(t, 4) for t in ms]} for g, (b, ms) in res.items()}


HEADLINE = dict(window=5, kind="ddf", p=0.25, dist="exact", M=4320, N=7680, phi=0.15, key=500)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prewarm-ms", type=float, default=200.0,
                    help="untimed back-to-back steps before the warm-up steps (ms)")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--forms", default="six_variants,large_frames,acwddf,effectiveness,batched,"
                                        "differentiable",
                    help="comma list of the form groups to run besides the step")
    ap.add_argument("--step-forms", default="loop,streams,direct",
                    help="forms of the six-variant DDF 3x3 group to time (comma list of loop, "
                         "streams, direct)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON tuning cache: applied instead of autotuning when the file exists, "
                         "written by the autotuner otherwise (fixes the tile shapes across runs, "
                         "e.g. between profiler passes)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one elementwise copy (float32 negation) of this many MiB, "
                         "untimed: the reference kernel for scaling HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build measures the single-GPU hot path "
              "(see the multi-GPU design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    groups = [g for g in args.forms.split(",") if g]
    known = ("six_variants", "large_frames", "acwddf", "effectiveness", "batched",
             "differentiable")
    if any(g not in known for g in groups):
        ap.error("--forms takes a comma list of " + ", ".join(known))
    forms_wanted = [f for f in args.step_forms.split(",") if f]
    if not forms_wanted or any(f not in ("loop", "streams", "direct") for f in forms_wanted):
        ap.error("--step-forms takes a comma list of loop, streams, direct")

    import torch
    from paper_1009_0958_amd import odf, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    DIST = {"exact": odf.EXACT, "minimax": odf.MINIMAX, "rgb": odf.RGB}
    global TUNE_CACHE, TUNE_CACHED
    TUNE_CACHE = args.tune_cache
    TUNE_CACHED = bool(TUNE_CACHE) and os.path.exists(TUNE_CACHE) and \
        os.path.getsize(TUNE_CACHE) > 0
    if TUNE_CACHED:
        with open(TUNE_CACHE) as f:
            for line in f:
                e = json.loads(line)
                if "window" in e:
                    TUNE_REPLAY.append((e["window"], e["kind"], e["dist"], e["u8"], e["config"]))

    # ---------------------------------------------------------------- the step
    # DDF 5x5 (p = 1/4, exact angle) on one 7680 x 4320 uint8 frame, correlated
    # impulsive noise 0.15: one launch of the forward per step, tile shape
    # chosen by the library's autotuner on this frame size first (untimed)
    H = HEADLINE
    M, N, w, p = H["M"], H["N"], H["window"], H["p"]
    img_np = synth.image_corr(M, N, H["phi"], key=H["key"])
    x = torch.from_numpy(img_np).to(dev)
    best_cfg, shape_ms = autotune(odf, w, odf.DDF, odf.EXACT, True, M, N, 3)
    out = torch.empty_like(x)
    idx = torch.empty((M, N), dtype=torch.uint8, device=dev)

    def step():
        odf.filter(x, w, odf.DDF, p, odf.EXACT, 4, out=out, idx=idx)

    # untimed: --prewarm-ms of back-to-back steps (the GPU's clock rises over
    # the first ~15 ms of sustained work: the first launches after the
    # autotuner's host work ran up to 20 % slower), then the W warm-up steps
    t_pre = time.perf_counter()
    while (time.perf_counter() - t_pre) * 1e3 < args.prewarm_ms:
        for _ in range(4):
            step()
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # events on the stream the filter launches on (torch's current stream)
    s_, e_ = _events(torch)
    t0 = time.perf_counter()
    s_.record()
    for _ in range(args.steps):
        step()
    e_.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = s_.elapsed_time(e_) / args.steps
    value = M * N / (ms_step * 1e3)
    ref_out, ref_idx = odf.filter(x, w, odf.DDF, p, odf.EXACT, 4)
    step_ok = bool(torch.equal(ref_out, out) and torch.equal(ref_idx, idx))

    ext = odf.tile_config(best_cfg)
    strip = best_cfg in (odf.STRIP, odf.SHORT_STRIP)
    slots_px = slots_per_pixel(w, "ddf", p, "exact")
    npx = M * N
    kname = ("fwd_strip_kernel<5, DDF, exact, uint8, %dx%d bands, " % tuple(ext)
             + ("8 bands per strip>" if best_cfg == odf.STRIP else "3 bands per strip>")
             if strip else "fwd_kernel<5, DDF, exact, uint8, %dx%d>" % tuple(ext))
    roofline = {
        "bound": "alu", "kernel": kname,
        "ms_per_launch": round(ms_step, 5),
        "achieved": round(slots_px * npx / (ms_step * 1e-3) / 1e12, 3),
        "peak": round(PEAK_SLOTS / 1e12, 2), "unit": "T VALU lane-slots/s",
        "frac": round(slots_px * npx / (ms_step * 1e-3) / PEAK_SLOTS, 4),
        "slots_per_pixel": slots_px, "pixels_per_launch": npx, "traffic": None,
        "hbm_bytes_per_pixel": 7, "hbm_frac": round(7 * npx / (ms_step * 1e-3) / 8e12, 5),
    }
    tb = traffic_bytes("ddf5_exact_7680x4320" + {odf.STRIP: "_strip", odf.SHORT_STRIP: "_strip3"}
                       .get(best_cfg, ""), ext)
    if tb is not None:
        roofline["traffic"] = tb["fetch"] + tb["write"]
        roofline["traffic_fetch_write"] = [tb["fetch"], tb["write"]]
        roofline["traffic_over_algorithmic"] = round((tb["fetch"] + tb["write"]) / (7 * npx), 3)

    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    forms = {}
    acw_idx = {}
    # seeded samples of the other forms' outputs, checked against the oracle in
    # the cpu_baseline leg (none when that leg is off)
    samples = None if args.no_cpu else {}
    if not args.no_forms:
        x1k_np = synth.image_corr(1024, 1024, 0.20)
        x1k = torch.from_numpy(x1k_np).to(dev)
        table = {
            "six_variants": lambda: six_variant_forms(torch, odf, dev, DIST, x1k, x1k_np, args,
                                                      forms_wanted, samples),
            "large_frames": lambda: large_frame_forms(torch, odf, synth, dev, DIST, samples),
            "acwddf": lambda: acwddf_forms(torch, odf, synth, dev, DIST, x1k, acw_idx),
            "effectiveness": lambda: effectiveness_forms(torch, odf, synth, dev, DIST),
            "batched": lambda: batched_form(torch, odf, synth, dev, DIST, samples),
            "differentiable": lambda: differentiable_forms(torch, odf, synth, dev)}
        for name in groups:
            t_form = time.perf_counter()
            try:
                forms.update(table[name]())
            except Exception as exc:  # keep the main line; report the failure
                forms[name + "_error"] = repr(exc)[:300]
            torch.cuda.empty_cache()
            print("bench: forms %s done (%.1f s)" % (name, time.perf_counter() - t_form),
                  file=sys.stderr, flush=True)
        if acw_idx:
            acw_idx["image"] = x1k_np

    print("bench: step %.4f ms, %.1f Mpixels/s" % (ms_step, value), file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(img_np, idx.cpu().numpy(), args.cpu_seconds, acw_idx, samples)

    line = {
        "metric": "Mpixels/s BVDF/DDF 3x3,5x5 fwd & fwd+bwd at 1 GPU; % roofline; mismatch rate",
        "value": round(value, 1), "unit": "Mpixels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "DDF 5x5 forward (p = 0.25, exact angle of eq. 2), one 7680x4320 "
                               "uint8 RGB frame: smooth field + 20 edges, correlated impulsive "
                               "noise 0.15; one launch per step",
                   "image": [M, N], "window": w, "p": p, "pair_term": "exact",
                   "launches_per_step": 1, "parallelism": "none"},
        "wall_s": round(wall, 3), "step_outputs_match_plain_launch": step_ok,
        "tuned": {"ddf5_exact_7680x4320": {"config": best_cfg, "ext_tile": ext,
                                          "ms_per_config": [round(t, 4) for t in shape_ms]}},
        "roofline": roofline, "forms": forms, "cpu_baseline": cpu,
        "paper_context": {"ddf3_exact_1024x1024_mpix_s": 0.0368,
                          "hardware": "Pentium D 2.66 GHz, C, gcc 3.4.4 (paper, Section II)"},
    }
    print(json.dumps(line), flush=True)


def six_variant_forms(torch, odf, dev, DIST, x, img_np, args, forms_wanted, samples):
    """DDF 3x3 on one 1024 x 1024 uint8 image (correlated impulsive noise 0.20)
    for p in {1/4, 1/2} x {exact, minimax q=4, rgb}: six forward filters,
    timed three ways (a loop of six launches; the six spread over three
    streams; the six as one planned batch recorded in a graph), with the
    per-variant kernel rates and the roofline of the fastest
    form's dominant kernel.  With ``samples`` the six index maps are kept for
    the oracle's full-image comparison."""
    M, N = img_np.shape[:2]
    variants = [(p, d) for p in (0.25, 0.5) for d in ("exact", "minimax", "rgb")]
    tuned = {}
    for d in ("exact", "minimax", "rgb"):
        best, times = autotune(odf, 3, odf.DDF, DIST[d], True, M, N, 10)
        tuned["ddf3_%s" % d] = {"config": best, "ext_tile": odf.tile_config(best),
                                "ms_per_config": [round(t, 5) for t in times]}
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

    graphs = {}
    batch_tuned = None
    if "direct" in forms_wanted:
        jobs = [dict(img=x, out=outs[(p, d)][0], idx=outs[(p, d)][1], window=3, kind=odf.DDF,
                     p=p, dist=DIST[d], q=4) for (p, d) in variants]
        batch_tuned = tune_batch(odf, jobs, "six_variants")
        plan = odf.BatchPlan(jobs)
        graphs["direct"] = (plan, plan.capture())

    step_forms = {}
    if "loop" in forms_wanted:
        step_forms["loop_of_launches"] = time_launches(torch, loop_step, args.steps, args.warmup)
    if "streams" in forms_wanted:
        step_forms["launches_on_3_streams"] = time_launches(torch, streams_step, args.steps,
                                                            args.warmup)
    for mode, (plan, g) in graphs.items():
        step_forms["graph_batch_" + mode] = time_launches(torch, g.replay, args.steps,
                                                          args.warmup)
    best = min(step_forms, key=step_forms.get)
    ms_step = step_forms[best]
    refs = {v: odf.filter(x, 3, odf.DDF, v[0], DIST[v[1]], 4) for v in variants}
    ok = True
    checked = ([loop_step] if "loop" in forms_wanted else []) + \
        ([streams_step] if "streams" in forms_wanted else [])
    for fn in checked + [g.replay for (_, g) in graphs.values()]:
        for o, i in outs.values():
            o.zero_()
            i.zero_()
        fn()
        torch.cuda.synchronize()
        ok = ok and all(torch.equal(refs[v][0], outs[v][0]) and torch.equal(refs[v][1], outs[v][1])
                        for v in variants)
    per_variant = {}
    for (p, d) in variants:
        o, i = outs[(p, d)]
        ms = time_launches(torch, lambda: odf.filter(x, 3, odf.DDF, p, DIST[d], 4, out=o, idx=i),
                           max(20, args.steps))
        slots = slots_per_pixel(3, "ddf", p, d) * M * N
        per_variant["ddf3_p%.2f_%s" % (p, d)] = {
            "ms": round(ms, 5), "mpix_s": round(M * N / (ms * 1e3), 1),
            "valu_frac": round(slots / (ms * 1e-3) / PEAK_SLOTS, 4)}
    npx = len(variants) * M * N
    slots_px = sum(slots_per_pixel(3, "ddf", p, d) for (p, d) in variants) / len(variants)
    if best == "graph_batch_direct":
        # one kernel over the tiles of all six variants: the form's time is its time
        info6 = graphs["direct"][0].info()
        ext6 = info6["ext_tiles"]["w3_ddf"]
        strip6 = info6["configs"][1] in (odf.STRIP, odf.SHORT_STRIP)
        dname = (("batch_strip_kernel ddf3 %dx%d bands" if strip6 else "batch_direct_kernel ddf3 %dx%d")
                 + ", six variants in one launch") % tuple(ext6)
        dms, dpx = ms_step, npx
        tb = None if strip6 else traffic_bytes("batch6", ext6)
    else:
        dom = max(per_variant, key=lambda k: per_variant[k]["ms"])
        dp, dd = float(dom.split("_")[1][1:]), dom.split("_")[2]
        dms, dpx = per_variant[dom]["ms"], M * N
        slots_px = slots_per_pixel(3, "ddf", dp, dd)
        dname = "fwd_kernel " + dom
        tb = traffic_bytes(dd, tuned["ddf3_%s" % dd]["ext_tile"])
    roof = {"bound": "alu", "kernel": dname, "ms_per_launch": round(dms, 5),
            "achieved": round(slots_px * dpx / (dms * 1e-3) / 1e12, 3),
            "peak": round(PEAK_SLOTS / 1e12, 2), "unit": "T VALU lane-slots/s",
            "frac": round(slots_px * dpx / (dms * 1e-3) / PEAK_SLOTS, 4),
            "slots_per_pixel": round(slots_px, 2), "pixels_per_launch": dpx, "traffic": None}
    if tb is not None:
        roof["traffic"] = tb["fetch"] + tb["write"]
        roof["traffic_over_algorithmic"] = round((tb["fetch"] + tb["write"]) / (7 * dpx), 3)
    if samples is not None:
        samples["six_variants"] = (img_np, {v: outs[v][1].cpu().numpy() for v in variants})
    return {"ddf3_six_variants_1024x1024": {
        "mpix_s": round(npx / (ms_step * 1e3), 1), "ms": round(ms_step, 5), "form": best,
        "forms_ms": {k: round(v, 5) for k, v in step_forms.items()},
        "outputs_match_plain_launch": ok, "tuned": tuned, "batch_tuned": batch_tuned,
        "variants": per_variant, "roofline": roof}}


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
    """7680 x 4320 frame (3x3 BVDF, 5x5, 7x7 and 9x9) and 64 x 1920 x 1080
    frames (5x5), correlated noise 0.15 (tile configs autotuned per class on a
    frame of this size first, untimed); 11x11 and 15x15 (the direct form) on
    one 1920 x 1080 frame.  With ``samples`` (a dict), the windows of 1 M seeded pixels
    (5x5; 100 000 for 3x3 and 7x7, 20 000 for 9x9) and the GPU's index there are
    kept for the oracle check of the cpu_baseline leg."""
    forms = {}
    for w, kk in ((3, odf.BVDF), (5, odf.BVDF), (5, odf.DDF), (7, odf.BVDF), (7, odf.DDF),
                  (9, odf.BVDF)):
        for d in ("exact", "minimax", "rgb"):
            if (w, kk, d) != (5, odf.DDF, "exact"):  # the step's class, tuned on this frame
                autotune(odf, w, kk, DIST[d], True, 4320, 7680, 3)
    # (9 x 9 DDF offers one config)
    for tag, shape, key in (("7680x4320", (1, 4320, 7680), 5), ("64x1920x1080", (64, 1080, 1920), 6)):
        B, M, N = shape
        imgs = np.stack([synth.image_corr(M, N, 0.15, key=key * 100 + b) for b in range(B)])
        big = torch.from_numpy(imgs).to(dev)
        del imgs
        bo = torch.empty_like(big)
        bi = torch.empty((B, M, N), dtype=torch.uint8, device=dev)
        npx = B * M * N
        for w, kind, p in ((3, "bvdf", 0.0), (5, "bvdf", 0.0), (5, "ddf", 0.25), (7, "bvdf", 0.0),
                           (7, "ddf", 0.25), (9, "bvdf", 0.0), (9, "ddf", 0.25)):
            if tag != "7680x4320" and w in (3, 7, 9):
                continue
            for d in ("exact", "minimax", "rgb"):
                kk = odf.BVDF if kind == "bvdf" else odf.DDF
                ms = time_launches(torch, lambda: odf.filter(big, w, kk, p, DIST[d], 4, out=bo,
                                                             idx=bi), 5, warm=1)
                name = "%s%d_%s_%s" % (kind, w, d, tag)
                forms[name] = {
                    "mpix_s": round(npx / (ms * 1e3), 1), "ms": round(ms, 3),
                    "config": odf.tune_get(w, kk, DIST[d], True),
                    "valu_frac": round(slots_per_pixel(w, kind, p, d) * npx / (ms * 1e-3)
                                       / PEAK_SLOTS, 4)}
                if samples is not None:
                    key = (tag, w)
                    if key not in samples.setdefault("windows", {}):
                        pix = mismatch_sample(B, M, N, {5: 1_000_000, 9: 20_000}.get(w, 100_000),
                                              7000 + 10 * w + key[0].count("x"))
                        samples["windows"][key] = (pix, sample_windows(torch, big, pix, w))
                    pix = samples["windows"][key][0]
                    gidx = bi.reshape(-1)[torch.from_numpy(pix).to(dev)].cpu().numpy()
                    samples.setdefault("cases", []).append((name, key, w, kind, p, d, gidx))
        del big, bo, bi
    # windows past 9x9 run the direct form (no configs; every pair term of a
    # window evaluated, n^2 per pixel): one 1920 x 1080 frame, exact angle
    img = torch.from_numpy(synth.image_corr(1080, 1920, 0.15, key=611)).to(dev)
    o = torch.empty_like(img)
    i = torch.empty((1080, 1920), dtype=torch.uint8, device=dev)
    for w in (11, 15):
        for kind, p in (("bvdf", 0.0), ("ddf", 0.25)):
            kk = odf.BVDF if kind == "bvdf" else odf.DDF
            ms = time_launches(torch, lambda: odf.filter(img, w, kk, p, odf.EXACT, 4, out=o, idx=i),
                               3, warm=1)
            # the cost model counts each unique pair once per pixel (what the
            # tile kernels evaluate); the direct form evaluates w^4 per pixel
            forms["%s%d_exact_1920x1080_direct" % (kind, w)] = {
                "mpix_s": round(1920 * 1080 / (ms * 1e3), 1), "ms": round(ms, 3),
                "pair_terms_per_px": w ** 4,
                "pair_terms_per_s": float("%.4g" % (1920 * 1080 * w ** 4 / (ms * 1e-3))),
                "unique_pair_model_frac": round(slots_per_pixel(w, kind, p, "exact") * 1920 * 1080
                                                / (ms * 1e-3) / PEAK_SLOTS, 4)}
    del img, o, i
    return forms


def acwddf_forms(torch, odf, synth, dev, DIST, x1k, acw_idx):
    """ACWDDF (lambda = 2, T = 10.8) on the 1024 x 1024 image and on a
    7680 x 4320 frame (3x3, 5x5 and 7x7), each pair term, configs tuned per size;
    the 1024 x 1024 3x3 index maps are kept for the oracle's mismatch count.
    Also CWVMF^2 and CWDDF^2 (exact) on the 1024 x 1024 image, tuned."""
    forms = {}
    big = torch.from_numpy(synth.image_corr(4320, 7680, 0.15, key=500)).to(dev)
    for w in (3, 5, 7):
        for d in ("exact", "minimax", "rgb"):
            for tag, img in (("1024x1024", x1k), ("7680x4320", big)):
                M, N = img.shape[:2]
                best, _ = autotune(odf, w, odf.ACWDDF, DIST[d], True, M, N, 5)
                o = torch.empty_like(img)
                i = torch.empty((M, N), dtype=torch.uint8, device=dev)
                ms = time_launches(torch, lambda: odf.acwddf(img, w, DIST[d], 4, 2, 10.8, out=o,
                                                             idx=i), 10, warm=2)
                forms["acwddf%d_%s_%s" % (w, d, tag)] = {
                    "mpix_s": round(M * N / (ms * 1e3), 1), "ms": round(ms, 4),
                    "config": best, "ext_tile": odf.tile_config(best),
                    "valu_frac": round(slots_per_pixel(w, "acw", 0.5, d) * M * N / (ms * 1e-3)
                                       / PEAK_SLOTS, 4),
                    "switched_to_ddf": round(float((i != (w * w - 1) // 2).float().mean()), 4)}
                if tag == "1024x1024" and w == 3:
                    acw_idx[d] = i.cpu().numpy()
    # the centre-weighted filters on their own (eq. 9), level k = 2, each on
    # the config its own table entry is tuned to
    M, N = x1k.shape[:2]
    o = torch.empty_like(x1k)
    i = torch.empty((M, N), dtype=torch.uint8, device=dev)
    for w in (3, 5, 7):
        for name, kind, d in (("cwvmf", odf.CWVMF, "rgb"), ("cwddf", odf.CWDDF, "exact")):
            best, _ = autotune(odf, w, kind, DIST[d], True, M, N, 5)
            ms = time_launches(torch, lambda: odf.cw_filter(x1k, w, kind, 2, DIST[d], 4, out=o,
                                                            idx=i), 10, warm=2)
            forms["%s%d_k2_1024x1024" % (name, w)] = {"mpix_s": round(M * N / (ms * 1e3), 1),
                                                      "ms": round(ms, 4), "config": best}
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


def batched_form(torch, odf, synth, dev, DIST, samples=None):
    """256 uint8 images of mixed size (64..2048 x 64..1536), window, kind and
    noise: one planned launch captured in a graph (one kernel per window and
    kind, on the tile shapes the batch autotuner picks per group on these
    jobs), against a
    loop of per-image launches of the same jobs (tile shapes from the per-image
    autotuner); also each group's jobs planned and replayed alone, whose
    summed times show how far the concurrent groups are from running back to
    back at their own rates."""
    specs = synth.mixed_batch_specs(256)
    imgs = synth.mixed_batch_images(specs, workers=16)
    # configs of the per-image launches of the loop, every class tuned on a
    # 1024 x 1024 image, about the batch's mean image size (untimed)
    tuned = {}
    for w in (3, 5):
        for kind in (odf.BVDF, odf.DDF):
            for d in ("exact", "minimax", "rgb"):
                best, _ = autotune(odf, w, kind, DIST[d], True, 1024, 1024, 5)
                tuned[f"w{w}_{'ddf' if kind else 'bvdf'}_{d}"] = best
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
    # the batch groups' tile shapes, tuned on these jobs (untimed)
    batch_tuned = tune_batch(odf, jobs, "batched")
    for j in jobs:
        j["out"].zero_()
        j["idx"].zero_()
    plan = odf.BatchPlan(jobs)
    graph = plan.capture()
    ms_direct = time_launches(torch, graph.replay, 5, warm=2)
    same = all(torch.equal(j["out"], o) and torch.equal(j["idx"], i)
               for j, (o, i) in zip(jobs, loop_out))
    info = plan.info()
    plan.close()
    alone = {}
    for w in (3, 5):
        for kind in (odf.BVDF, odf.DDF):
            sub = [j for j in jobs if j["window"] == w and j["kind"] == kind]
            gp = odf.BatchPlan(sub)
            gg = gp.capture()
            alone[f"w{w}_{'ddf' if kind else 'bvdf'}"] = {
                "mpix": round(sum(int(j["img"].shape[0] * j["img"].shape[1]) for j in sub) / 1e6,
                              2),
                "ms": round(time_launches(torch, gg.replay, 5, warm=2), 3)}
            gp.close()
    if samples is not None:
        # 1 M seeded pixels over the whole batch (the outputs of the last
        # replay of the group graphs, bitwise equal to the whole plan's)
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
    return {"batched_256_mixed": {
        "mpix": round(npx / 1e6, 2), "loop_configs": tuned,
        "batch_tile_shapes": batch_tuned, "plan_ext_tiles": info["ext_tiles"],
        "plan_configs": dict(zip(("w3_bvdf", "w3_ddf", "w5_bvdf", "w5_ddf", "w7_bvdf", "w7_ddf",
                                  "w9_bvdf", "w9_ddf"),
                                 info["configs"])),
        "direct_graph_ms": round(ms_direct, 3),
        "direct_graph_mpix_s": round(npx / (ms_direct * 1e3), 1),
        "loop_ms": round(ms_loop, 3), "loop_mpix_s": round(npx / (ms_loop * 1e3), 1),
        "speedup_direct_vs_loop": round(ms_loop / ms_direct, 3),
        "groups_alone": alone,
        "groups_alone_sum_ms": round(sum(v["ms"] for v in alone.values()), 3),
        "bitwise_equal_to_loop": bool(same), "tiles_per_class": info["tiles"]}}


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
    softmin fwd + bwd at tau 0.01 and 0.1 (and 7x7 at tau 0.1); a plain PyTorch
    softmin on 2 of the images for comparison."""
    forms = {}
    x = torch.from_numpy(synth.float_batch(16, 512, 512, 0.1)).to(dev)
    dy = torch.randn_like(x)
    npx = 16 * 512 * 512
    out = torch.empty_like(x)
    idx = torch.empty(x.shape[:3], dtype=torch.uint8, device=dev)
    # the hard forward's config, tuned on a float32 frame of the batch's rows and pixel count
    hard_cfg, _ = autotune(odf, 5, odf.DDF, odf.EXACT, False, 512, 8192, 3)
    ms_f = time_launches(torch, lambda: odf.filter(x, 5, odf.DDF, 0.25, odf.EXACT, 4, out=out,
                                                   idx=idx), 10)
    ms_b = time_launches(torch, lambda: odf.backward_hard(idx, dy, 5), 10)
    forms["ddf5_f32_16x512x512_hard"] = {
        "fwd_ms": round(ms_f, 3), "bwd_ms": round(ms_b, 3), "fwd_config": hard_cfg,
        "fwd_bwd_mpix_s": round(npx / ((ms_f + ms_b) * 1e3), 1),
        "fwd_valu_frac": round(slots_per_pixel(5, "ddf", 0.25, "exact", u8=False) * npx
                               / (ms_f * 1e-3)
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
    ws7 = torch.empty(odf.lib().odf_softmin_bwd_workspace(16, 512, 512, 7, odf.DDF),
                      dtype=torch.uint8, device=dev)
    ms_sf = time_launches(torch, lambda: odf.softmin_forward(x, 7, odf.DDF, 0.25, 0.1), 3)
    ms_sb = time_launches(torch, lambda: odf.softmin_backward(x, dy, 7, odf.DDF, 0.25, 0.1,
                                                              workspace=ws7), 3)
    del ws7
    forms["ddf7_f32_16x512x512_softmin_tau0.1"] = {
        "fwd_ms": round(ms_sf, 3), "bwd_ms": round(ms_sb, 3),
        "fwd_bwd_mpix_s": round(npx / ((ms_sf + ms_sb) * 1e3), 1),
        "fwd_valu_frac": round(softmin_slots_per_pixel(7, False) * npx / (ms_sf * 1e-3)
                               / PEAK_SLOTS, 4),
        "bwd_valu_frac": round(softmin_slots_per_pixel(7, True) * npx / (ms_sb * 1e-3)
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


def acwddf_mismatch(oracle, acw_idx, codes, k=20000):
    """ACWDDF 3x3 index mismatches against the oracle on k seeded pixels of the
    1024 x 1024 image, and whether each one is undetermined at binary32
    precision (S within 1e-5 of T, or a near-tie within 1e-6 between members of
    different colours in one of the four selections)."""
    img_np = acw_idx["image"]
    M, N = img_np.shape[:2]
    pix = np.sort(np.random.default_rng(1010).choice(M * N, k, replace=False))
    rr, cc = pix // N, pix % N
    cols = np.stack([img_np[np.clip(rr + u // 3 - 1, 0, M - 1), np.clip(cc + u % 3 - 1, 0, N - 1)]
                     for u in range(9)], axis=1)
    res = {}
    for d, g_idx in acw_idx.items():
        if d == "image":
            continue
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


def mismatch_report(cols, g, O):
    """Mismatches of the GPU's indices g (k,) against the oracle's objectives O
    (k, n) of the same windows, whose member colours are cols (k, n, 3):
    their count, whether each is a near-tie (the oracle's objective of the
    GPU's choice within 1e-6 relative of the minimum), and a breakdown by the
    two members' colours: collinear (one a positive multiple of the other:
    eq. 2 gives them the same angle to every pixel) or not, and whether the
    oracle's two objectives tie exactly in binary64."""
    k = O.shape[0]
    rows = np.arange(k)
    first = O.argmin(1)
    diff = g != first
    og = O[rows, g]
    omin = O.min(1)
    near = (og <= omin * (1 + 1e-6)) | ((omin == 0) & (og == 0))
    a = cols[rows, g][diff].astype(np.int64)
    b = cols[rows, first][diff].astype(np.int64)
    collinear = np.all(np.cross(a, b) == 0, axis=1)
    exact = og[diff] == omin[diff]
    return {"index_mismatch": int(diff.sum()), "index_compared": int(k),
            "mismatches_all_near_ties": bool(np.all(near[diff])),
            "collinear_exact_tie": int((collinear & exact).sum()),
            "collinear_inexact": int((collinear & ~exact).sum()),
            "noncollinear_exact_tie": int((~collinear & exact).sum()),
            "noncollinear_inexact": int((~collinear & ~exact).sum())}


def sampled_mismatch(oracle, samples, codes):
    """Index mismatches of the kept samples against the oracle, per form (each
    sampled pixel's window given to the oracle as a w x w patch of its own),
    with the near-tie check and breakdown of mismatch_report; the six DDF 3x3
    variants on the whole 1024 x 1024 image."""
    def check(win, gidx, w, kind, p, d):
        k = win.shape[0]
        centre = np.arange(k) * w * w + (w * w) // 2
        _, _, _, _, O = oracle.filter_at(win, centre, w, kind, p, codes[d])
        return mismatch_report(win.reshape(k, w * w, 3), gidx.astype(np.int64), O)

    res = {}
    t0 = time.perf_counter()
    if "six_variants" in samples:
        img_np, maps = samples["six_variants"]
        M, N = img_np.shape[:2]
        pix = np.arange(M * N)
        rr, cc = pix // N, pix % N
        cols = np.stack([img_np[np.clip(rr + u // 3 - 1, 0, M - 1),
                                np.clip(cc + u % 3 - 1, 0, N - 1)] for u in range(9)], axis=1)
        for (p, d), gmap in maps.items():
            _, _, _, _, O = oracle.filter_at(img_np, pix, 3, oracle.DDF, p, codes[d])
            res["ddf3_p%.2f_%s_1024x1024" % (p, d)] = mismatch_report(
                cols, gmap.reshape(-1).astype(np.int64), O)
    for name, key, w, kind, p, d, gidx in samples.get("cases", []):
        win = samples["windows"][key][1]
        res[name] = check(win, gidx, w, oracle.DDF if kind == "ddf" else oracle.BVDF, p, d)
    if samples.get("batch"):
        tot = None
        for w, kind, p, win, gidx in samples["batch"]:
            r = check(win, gidx, w, kind, p, "exact")
            if tot is None:
                tot = r
            else:
                for f, v in r.items():
                    tot[f] = (tot[f] and v) if isinstance(v, bool) else tot[f] + v
        res["batched_256_mixed"] = tot
    res["seconds"] = round(time.perf_counter() - t0, 1)
    return res


def cpu_baseline(img_np, gidx, seconds, acw_idx=None, samples=None):
    """The FP64 oracle on a band of whole rows of the step's frame (DDF 5x5,
    p = 1/4, exact), all host threads, sized to about ``seconds``; the GPU's
    index mismatches on that band (near-ties only, with their breakdown); and
    the index mismatches of the kept samples of the other forms."""
    import oracle

    H = HEADLINE
    M, N, w, p = H["M"], H["N"], H["window"], H["p"]
    h = w // 2

    def band(r0, rows):
        """The oracle's selection on rows [r0, r0 + rows): the band with h
        rows of halo each side (the frame's own border where it ends)."""
        lo, hi = max(0, r0 - h), min(M, r0 + rows + h)
        _, o_idx = oracle.filter(img_np[lo:hi], w, oracle.DDF, p, oracle.EXACT)
        return o_idx[r0 - lo:r0 - lo + rows]

    t0 = time.perf_counter()
    band(0, 8)
    per_px = (time.perf_counter() - t0) / (8 * N)
    rows = int(min(M, max(8, seconds / (per_px * N))))
    r0 = (M - rows) // 2
    t0 = time.perf_counter()
    o_idx = band(r0, rows)
    dt = time.perf_counter() - t0
    g = gidx[r0:r0 + rows].astype(np.int64).reshape(-1)
    pix = np.arange(r0 * N, (r0 + rows) * N)
    diff = np.nonzero(g != o_idx.reshape(-1))[0]
    report = {"index_mismatch": 0, "index_compared": int(g.size), "mismatches_all_near_ties": True}
    if diff.size:
        _, _, _, _, O = oracle.filter_at(img_np, pix[diff], w, oracle.DDF, p, oracle.EXACT)
        rr, cc = pix[diff] // N, pix[diff] % N
        cols = np.stack([img_np[np.clip(rr + u // w - h, 0, M - 1),
                                np.clip(cc + u % w - h, 0, N - 1)] for u in range(w * w)], axis=1)
        report = mismatch_report(cols, g[diff], O)
        report["index_compared"] = int(g.size)
    codes = {"exact": 0, "minimax": 1, "rgb": 2}
    return {"value": round(rows * N / dt / 1e6, 5), "unit": "Mpixels/s",
            "cores": oracle.threads(), "cpu_model": host_cpu_model(), "kind": "oracle",
            "sample": "rows %d..%d (%d x %d pixels) of the 7680x4320 frame, DDF 5x5 p=0.25 "
                      "exact, whole-band oracle pass (%.1f s)" % (r0, r0 + rows - 1, rows, N, dt),
            **report,
            "acwddf3_1024x1024": acwddf_mismatch(oracle, acw_idx, codes) if acw_idx else None,
            "forms_mismatch": sampled_mismatch(oracle, samples, codes) if samples else None}


if __name__ == "__main__":
    main()
