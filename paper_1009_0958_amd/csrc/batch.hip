// batch.hip -- many uint8 images of different sizes, windows and filter
// variants in one launch per kernel group.
//
// odf_batch_plan cuts every job into output tiles and uploads one work list
// per group (window, kind): the tiles of every pair term of that window and
// kind, larger tiles first.  A group kernel takes each tile's pair term from
// its job and runs the matching tile function (a uniform branch), so a plan
// of many small images or several variants of one image fills the GPU with
// one grid instead of a few short ones and their tails.  The pair-term
// variants of one window share a register budget (3x3: 64 VGPRs); windows
// and kinds do not (a kernel branching over 3x3 and 5x5 would carry the 5x5
// budget everywhere), so they keep kernels of their own.  Each group runs one
// workgroup per tile of its list, dispatched in list order, on the config of
// the batch tuning table: one of the four extended tile shapes, or the strip
// form, whose work items are 32-wide strips of 8 (or 3) bands that keep the
// rows shared by consecutive bands in LDS (fwd_strip.h); odf_autotune_batch
// times the six on a mixed list, odf_autotune_batch_jobs on the caller's jobs.  odf_batch_launch enqueues the group kernels,
// forked onto per-plan auxiliary streams (default priority) and joined back
// with events so that groups run concurrently and their tails overlap; it
// allocates nothing and never synchronises, so it can be captured in a
// hipGraph.  Every tile or strip writes only its own outputs with the same
// function as the per-image kernels, so results do not depend on the config
// or on which workgroup takes which item.
#include <stdio.h>

#include <algorithm>
#include <new>
#include <vector>

#include "fwd_strip.h"
#include "odf.h"

namespace odf {

struct BatchJob {
    const uint8_t* img;
    uint8_t* out;
    uint8_t* idx;
    int M, N;
    int dist;
    float p;
    MinimaxCoef coef;
};

struct BatchTile {
    int job;
    int ty0, tx0;
};

struct BatchClass {
    const BatchJob* jobs;
    const BatchTile* tiles;
    int ntiles;
    int bands;  // strip form: bands per strip
};

// Extended-tile shape CFG of the batch kernels: the per-image table's shapes.
template <int CFG>
struct BatchShape {
    static constexpr int EXT_W = kTileW[CFG];
    static constexpr int EXT_H = kTileH[CFG];
    static constexpr int THREADS = EXT_W * EXT_H;
};

constexpr int kNumClasses = 3 * kNumBatchGroups;  // (window 3/5/7/9) x (BVDF/DDF) x (exact/minimax/rgb)

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
template <typename T>
__device__ __forceinline__ T* uni(T* v) {
    const uint64_t a = reinterpret_cast<uint64_t>(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// Filter tile t of a group work list (all fields are uniform over the
// workgroup and are moved to scalar registers).
template <int W, int KIND, int DIST, int CFG>
__device__ __forceinline__ void batch_tile(
    FwdSharedFor<W, KIND, DIST, true, BatchShape<CFG>::EXT_W, BatchShape<CFG>::EXT_H, false>& sh,
    const BatchClass& bc, const BatchTile& tile) {
    constexpr int EXT_W = BatchShape<CFG>::EXT_W, EXT_H = BatchShape<CFG>::EXT_H;
    const BatchJob& job = bc.jobs[uni(tile.job)];
    FwdParams prm{};
    prm.img = uni(job.img);
    prm.out = uni(job.out);
    prm.idx = uni(job.idx);
    prm.B = 1;
    prm.M = uni(job.M);
    prm.N = uni(job.N);
    prm.p = uni(job.p);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        prm.coef.asin_c[k] = uni(job.coef.asin_c[k]);
        prm.coef.acos_c[k] = uni(job.coef.acos_c[k]);
    }
    fwd_tile<W, KIND, DIST, true, EXT_W, EXT_H, false>(sh, prm, 0, uni(tile.ty0), uni(tile.tx0),
                                                       threadIdx.x);
}

// LDS of a group kernel: room for the tile of any pair term.
template <int W, int KIND, int CFG>
struct BatchSmem {
    template <int DIST>
    using Sh = FwdSharedFor<W, KIND, DIST, true, BatchShape<CFG>::EXT_W,
                            BatchShape<CFG>::EXT_H, false>;
    static constexpr size_t a = sizeof(Sh<kExact>), b = sizeof(Sh<kMinimax>),
                            c = sizeof(Sh<kRgb>);
    static constexpr size_t BYTES = a > b ? (a > c ? a : c) : (b > c ? b : c);
};

// One workgroup per tile of the list, dispatched in list order; the tile's
// pair term comes from its job (uniform branch).  The register targets are
// the per-image kernels' for 3x3 (64 VGPRs); the 5x5 groups hold all three
// pair terms, whose budgets differ, and take none.
template <int W, int KIND, int CFG>
__global__ void __launch_bounds__(BatchShape<CFG>::THREADS)
    __attribute__((amdgpu_waves_per_eu(W == 3 ? 8 : 1))) batch_direct_kernel(BatchClass bc) {
    __shared__ __align__(16) char smem[BatchSmem<W, KIND, CFG>::BYTES];
    const int t = flat_block(bc.ntiles);
    if (t < 0) return;
    const BatchTile tile = bc.tiles[t];
    const int dist = uni(bc.jobs[uni(tile.job)].dist);
    using S = BatchSmem<W, KIND, CFG>;
    if (dist == kExact)
        batch_tile<W, KIND, kExact, CFG>(*reinterpret_cast<typename S::template Sh<kExact>*>(smem),
                                         bc, tile);
    else if (dist == kMinimax)
        batch_tile<W, KIND, kMinimax, CFG>(
            *reinterpret_cast<typename S::template Sh<kMinimax>*>(smem), bc, tile);
    else
        batch_tile<W, KIND, kRgb, CFG>(*reinterpret_cast<typename S::template Sh<kRgb>*>(smem),
                                       bc, tile);
}

// The strip form of a group (configs kStripConfig, kShortStripConfig): one
// workgroup per strip of the list (ty0, tx0 its first output row and column),
// 32-wide strips of bands of 16 rows as in the per-image strip kernels.
template <int W, int KIND, int DIST>
using StripSh = StripShared<W, KIND, DIST, true, 32, 16>;

template <int W, int KIND>
struct BatchStripSmem {
    static constexpr size_t a = sizeof(StripSh<W, KIND, kExact>),
                            b = sizeof(StripSh<W, KIND, kMinimax>),
                            c = sizeof(StripSh<W, KIND, kRgb>);
    static constexpr size_t BYTES = a > b ? (a > c ? a : c) : (b > c ? b : c);
};

template <int W, int KIND, int DIST>
__device__ __forceinline__ void batch_strip(StripSh<W, KIND, DIST>& sh, const BatchClass& bc,
                                            const BatchTile& tile) {
    const BatchJob& job = bc.jobs[uni(tile.job)];
    FwdParams prm{};
    prm.img = uni(job.img);
    prm.out = uni(job.out);
    prm.idx = uni(job.idx);
    prm.B = 1;
    prm.M = uni(job.M);
    prm.N = uni(job.N);
    prm.p = uni(job.p);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        prm.coef.asin_c[k] = uni(job.coef.asin_c[k]);
        prm.coef.acos_c[k] = uni(job.coef.acos_c[k]);
    }
    fwd_strip<W, KIND, DIST, true, 32, 16>(sh, prm, 0, uni(tile.ty0), uni(tile.tx0), uni(bc.bands));
}

// Occupancy target: the waves per SIMD the LDS of the largest pair term allows.
template <int W, int KIND>
__global__ void __launch_bounds__(512)
    __attribute__((amdgpu_waves_per_eu(lds_waves_per_eu(BatchStripSmem<W, KIND>::BYTES, 512))))
    batch_strip_kernel(BatchClass bc) {
    __shared__ __align__(16) char smem[BatchStripSmem<W, KIND>::BYTES];
    const int t = flat_block(bc.ntiles);
    if (t < 0) return;
    const BatchTile tile = bc.tiles[t];
    const int dist = uni(bc.jobs[uni(tile.job)].dist);
    if (dist == kExact)
        batch_strip<W, KIND, kExact>(*reinterpret_cast<StripSh<W, KIND, kExact>*>(smem), bc, tile);
    else if (dist == kMinimax)
        batch_strip<W, KIND, kMinimax>(*reinterpret_cast<StripSh<W, KIND, kMinimax>*>(smem), bc,
                                       tile);
    else
        batch_strip<W, KIND, kRgb>(*reinterpret_cast<StripSh<W, KIND, kRgb>*>(smem), bc, tile);
}

// class = batch_group(window, kind) * 3 + dist; group = class / 3
constexpr int kNumGroups = kNumBatchGroups;
static int group_window(int grp) { return batch_group_window(grp); }

static void group_geometry(int grp, int cfg, int& tw, int& th, int& threads) {
    const int h = group_window(grp) / 2;
    if (is_strip_config(cfg)) {
        tw = 32 - 2 * h;
        th = strip_bands(cfg) * 16 - 2 * h;
        threads = 512;
        return;
    }
    tw = kTileW[cfg] - 2 * h;
    th = kTileH[cfg] - 2 * h;
    threads = kTileW[cfg] * kTileH[cfg];
}

// (7x7 groups offer the 512-thread shapes 2 and 3 and the strips, 9x9 groups
// shape 2 and, for BVDF, the strips, as the per-image kernels do; make_plan
// rejects the others)
template <int W, int KIND>
static void launch_group_wk(int cfg, int threads, const BatchClass& bc, hipStream_t s) {
    const dim3 grid = flat_grid(bc.ntiles);
    switch (cfg) {
    case 0:
        if constexpr (W < 7)
            hipLaunchKernelGGL((batch_direct_kernel<W, KIND, 0>), grid, dim3(threads), 0, s, bc);
        break;
    case 1:
        if constexpr (W < 7)
            hipLaunchKernelGGL((batch_direct_kernel<W, KIND, 1>), grid, dim3(threads), 0, s, bc);
        break;
    case 2: hipLaunchKernelGGL((batch_direct_kernel<W, KIND, 2>), grid, dim3(threads), 0, s, bc); break;
    case 3:
        if constexpr (W < 9)
            hipLaunchKernelGGL((batch_direct_kernel<W, KIND, 3>), grid, dim3(threads), 0, s, bc);
        break;
    default:
        if constexpr (strip_form<W, KIND, true>())
            hipLaunchKernelGGL((batch_strip_kernel<W, KIND>), grid, dim3(threads), 0, s, bc);
        break;
    }
}

static void launch_group(int grp, int cfg, int threads, const BatchClass& bc, hipStream_t s) {
    switch (grp) {
    case 0: launch_group_wk<3, kBVDF>(cfg, threads, bc, s); break;
    case 1: launch_group_wk<3, kDDF>(cfg, threads, bc, s); break;
    case 2: launch_group_wk<5, kBVDF>(cfg, threads, bc, s); break;
    case 3: launch_group_wk<5, kDDF>(cfg, threads, bc, s); break;
    case 4: launch_group_wk<7, kBVDF>(cfg, threads, bc, s); break;
    case 5: launch_group_wk<7, kDDF>(cfg, threads, bc, s); break;
    case 6: launch_group_wk<9, kBVDF>(cfg, threads, bc, s); break;
    default: launch_group_wk<9, kDDF>(cfg, threads, bc, s); break;
    }
}

}  // namespace odf

// Opaque plan (declared in odf.h).
struct odf_plan {
    odf::BatchJob* d_jobs = nullptr;
    odf::BatchTile* d_tiles = nullptr;
    int class_tiles[odf::kNumClasses] = {};  // per class, for odf_plan_info
    int ntiles[odf::kNumGroups] = {};
    int offset[odf::kNumGroups] = {};
    int cfg[odf::kNumGroups] = {};  // tile shape of each group
    int njobs = 0;
    long long npix = 0;
    hipStream_t aux[odf::kNumGroups] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[odf::kNumGroups] = {};
};

namespace {

int bfail(int code, const char* msg) { return odf::set_error(code, "%s", msg); }

// Relative cost of a tile pixel per pair term (3x3 DDF instruction counts),
// used to put the heaviest tiles first.
int dist_weight(int dist) { return dist == ODF_MINIMAX ? 13 : (dist == ODF_EXACT ? 12 : 10); }

void destroy(odf_plan* p) {
    if (!p) return;
    for (int g = 0; g < odf::kNumGroups; ++g) {
        if (p->aux[g]) (void)hipStreamDestroy(p->aux[g]);
        if (p->join[g]) (void)hipEventDestroy(p->join[g]);
    }
    if (p->fork) (void)hipEventDestroy(p->fork);
    (void)hipFree(p->d_jobs);
    (void)hipFree(p->d_tiles);
    delete p;
}

// Validate the jobs and build a plan whose groups run on the tile shapes cfg
// (one per group).
int make_plan(const odf_job* jobs, int njobs, const int* cfg, odf_plan** plan) {
    if (!plan) return bfail(ODF_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (!jobs || njobs < 1) return bfail(ODF_EINVAL, "jobs must be a non-empty array");
    std::vector<odf::BatchJob> hj(njobs);
    for (int i = 0; i < njobs; ++i) {
        const odf_job& j = jobs[i];
        if (!j.img || !j.out) return bfail(ODF_EINVAL, "job img/out is NULL");
        if (j.M < 1 || j.N < 1 || (long long)j.M * j.N >= (1ll << 31))
            return bfail(ODF_EINVAL, "job size out of range");
        if (!odf::batch_window(j.window))
            return bfail(ODF_EUNSUPPORTED, "job window not 3, 5, 7 or 9");
        if (j.kind != ODF_BVDF && j.kind != ODF_DDF) return bfail(ODF_EINVAL, "job kind out of range");
        if (j.dist < ODF_EXACT || j.dist > ODF_RGB) return bfail(ODF_EINVAL, "job dist out of range");
        if (j.dist == ODF_MINIMAX && (j.q < 2 || j.q > 4)) return bfail(ODF_EINVAL, "job q out of range");
        if (j.kind == ODF_DDF && !(j.p >= 0.0f && j.p <= 1.0f)) return bfail(ODF_EINVAL, "job p out of range");
        const size_t nb = (size_t)j.M * j.N * 3;
        const char* a = (const char*)j.img;
        const char* o = (const char*)j.out;
        if (a < o + nb && o < a + nb) return bfail(ODF_EINVAL, "job out overlaps img");
    }

    // (cost, tile) per group; cost = output pixels x pair-term weight
    std::vector<std::pair<long long, odf::BatchTile>> lists[odf::kNumGroups];
    int class_tiles[odf::kNumClasses] = {};
    long long npix = 0, total_tiles = 0;
    for (int i = 0; i < njobs; ++i) {
        const odf_job& j = jobs[i];
        odf::BatchJob& b = hj[i];
        b.img = j.img;
        b.out = j.out;
        b.idx = j.idx;
        b.M = j.M;
        b.N = j.N;
        b.dist = j.dist;
        b.p = j.kind == ODF_DDF ? j.p : 0.0f;
        b.coef = odf::MinimaxCoef{};
        if (j.dist == ODF_MINIMAX) b.coef = odf::minimax_coef(j.q);
        const int grp = odf::batch_group(j.window, j.kind);
        if (!odf::tile_config_valid(j.window, j.kind, cfg[grp], true))
            return bfail(ODF_EINVAL, "config not offered for a job's window and kind");
        int tw, th, thr;
        odf::group_geometry(grp, cfg[grp], tw, th, thr);
        for (int ty = 0; ty < j.M; ty += th)
            for (int tx = 0; tx < j.N; tx += tw) {
                const long long cost = (long long)std::min(th, j.M - ty) * std::min(tw, j.N - tx) *
                                       dist_weight(j.dist);
                if (++total_tiles >= INT32_MAX)  // tile ids and list offsets are int
                    return bfail(ODF_EINVAL, "the batch has 2^31 - 1 tiles or more");
                lists[grp].push_back({cost, odf::BatchTile{i, ty, tx}});
                ++class_tiles[grp * 3 + j.dist];
            }
        npix += (long long)j.M * j.N;
    }
    odf_plan* p = odf::test_fail_alloc() ? nullptr : new (std::nothrow) odf_plan;
    if (!p) return bfail(ODF_ENOMEM, "plan allocation failed");
    for (int c = 0; c < odf::kNumClasses; ++c) p->class_tiles[c] = class_tiles[c];
    std::vector<odf::BatchTile> all;
    for (int g = 0; g < odf::kNumGroups; ++g) {
        std::stable_sort(lists[g].begin(), lists[g].end(),
                         [](const std::pair<long long, odf::BatchTile>& x,
                            const std::pair<long long, odf::BatchTile>& y) { return x.first > y.first; });
        p->offset[g] = (int)all.size();
        p->ntiles[g] = (int)lists[g].size();
        p->cfg[g] = cfg[g];
        for (auto& t : lists[g]) all.push_back(t.second);
    }
    if (hipMalloc(&p->d_jobs, sizeof(odf::BatchJob) * hj.size()) != hipSuccess ||
        hipMalloc(&p->d_tiles, sizeof(odf::BatchTile) * std::max<size_t>(1, all.size())) != hipSuccess) {
        destroy(p);
        return bfail(ODF_ENOMEM, "device allocation for the plan failed");
    }
    if (hipMemcpy(p->d_jobs, hj.data(), sizeof(odf::BatchJob) * hj.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->d_tiles, all.data(), sizeof(odf::BatchTile) * all.size(), hipMemcpyHostToDevice) !=
            hipSuccess) {
        destroy(p);
        return bfail(ODF_EHIP, "uploading the plan failed");
    }
    // auxiliary streams for every non-empty group after the first
    bool first = true;
    for (int g = 0; g < odf::kNumGroups; ++g) {
        if (p->ntiles[g] == 0) continue;
        if (first) { first = false; continue; }
        if (hipStreamCreateWithFlags(&p->aux[g], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->join[g], hipEventDisableTiming) != hipSuccess) {
            destroy(p);
            return bfail(ODF_EHIP, "creating the plan's streams failed");
        }
    }
    if (hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess) {
        destroy(p);
        return bfail(ODF_EHIP, "creating the plan's events failed");
    }
    p->njobs = njobs;
    p->npix = npix;
    *plan = p;
    return ODF_OK;
}

// Time the six configs (four tile shapes, two strip heights) of group grp on the
// jobs of that group among jobs[] (reps launches each after two untimed ones);
// ms[c] = -1 when the group has no job.  Returns ODF_OK or an error code (message set).
int time_group_shapes(const odf_job* jobs, int njobs, int grp, int reps, float* ms,
                      hipStream_t s) {
    std::vector<odf_job> sub;
    for (int i = 0; i < njobs; ++i)
        if (odf::batch_group(jobs[i].window, jobs[i].kind) == grp) sub.push_back(jobs[i]);
    for (int c = 0; c < odf::kNumTileConfigs; ++c) ms[c] = -1.0f;
    if (sub.empty()) return ODF_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return bfail(ODF_EHIP, "autotune_batch: event creation failed");
    }
    int rc = ODF_OK;
    for (int c = 0; c < odf::kNumTileConfigs && rc == ODF_OK; ++c) {
        if (!odf::tile_config_valid(odf::group_window(grp), grp % 2, c, true)) continue;  // -1
        int cfg[odf::kNumGroups];
        for (int g = 0; g < odf::kNumGroups; ++g) cfg[g] = odf::batch_tuned_config(g);
        cfg[grp] = c;
        odf_plan* plan = nullptr;
        rc = make_plan(sub.data(), (int)sub.size(), cfg, &plan);
        if (rc != ODF_OK) break;
        bool ok = odf_batch_launch(plan, s) == ODF_OK && odf_batch_launch(plan, s) == ODF_OK &&
                  hipEventRecord(e0, s) == hipSuccess;
        for (int r = 0; r < reps; ++r) ok = ok && odf_batch_launch(plan, s) == ODF_OK;
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float t = 0.0f;
        ok = ok && hipEventElapsedTime(&t, e0, e1) == hipSuccess;
        destroy(plan);
        if (!ok) rc = bfail(ODF_EHIP, "autotune_batch: timing failed");
        else ms[c] = t / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// The fastest config of ms[kNumTileConfigs] (ignoring -1), or -1.
int fastest(const float* ms) {
    int best = -1;
    for (int c = 0; c < odf::kNumTileConfigs; ++c)
        if (ms[c] >= 0.0f && (best < 0 || ms[c] < ms[best])) best = c;
    return best;
}

// Append the batch tuning line of group grp to cache_path.
int write_batch_line(const char* cache_path, int grp, int best, const float* ms) {
    if (!cache_path) return ODF_OK;
    hipDeviceProp_t prop;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return bfail(ODF_EHIP, "autotune_batch: device query failed");
    FILE* f = fopen(cache_path, "a");
    if (!f) return odf::set_error(ODF_EINVAL, "cannot open %s", cache_path);
    fprintf(f,
            "{\"arch\": \"%s\", \"batch_window\": %d, \"kind\": %d, \"config\": %d, "
            "\"ms\": [%.5f, %.5f, %.5f, %.5f, %.5f, %.5f]}\n",
            prop.gcnArchName, odf::group_window(grp), grp % 2, best, ms[0], ms[1], ms[2], ms[3],
            ms[4], ms[5]);
    fclose(f);
    return ODF_OK;
}

}  // namespace

extern "C" {

int odf_batch_plan(const odf_job* jobs, int njobs, odf_plan** plan, void* stream) {
    (void)stream;
    int cfg[odf::kNumGroups];
    for (int g = 0; g < odf::kNumGroups; ++g) cfg[g] = odf::batch_tuned_config(g);
    return make_plan(jobs, njobs, cfg, plan);
}

int odf_batch_plan_ex(const odf_job* jobs, int njobs, int flags, odf_plan** plan, void* stream) {
    if (plan) *plan = nullptr;
    if (flags == ODF_BATCH_PERSISTENT)
        return bfail(ODF_EUNSUPPORTED,
                     "the persistent batch form is retired: the direct form runs the groups at "
                     "the kernels' own steady-state rate");
    if (flags != ODF_BATCH_DIRECT) return bfail(ODF_EINVAL, "flags must be ODF_BATCH_DIRECT");
    return odf_batch_plan(jobs, njobs, plan, stream);
}

int odf_batch_launch(const odf_plan* plan, void* stream) {
    if (!plan) return bfail(ODF_EINVAL, "plan is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipEventRecord(plan->fork, s) != hipSuccess) return bfail(ODF_EHIP, "fork event failed");
    for (int g = 0; g < odf::kNumGroups; ++g) {
        if (plan->ntiles[g] == 0) continue;
        odf::BatchClass bc{plan->d_jobs, plan->d_tiles + plan->offset[g], plan->ntiles[g],
                           odf::strip_bands(plan->cfg[g])};
        int tw, th, thr;
        odf::group_geometry(g, plan->cfg[g], tw, th, thr);
        hipStream_t cs = plan->aux[g] ? plan->aux[g] : s;
        if (cs != s && hipStreamWaitEvent(cs, plan->fork, 0) != hipSuccess)
            return bfail(ODF_EHIP, "stream fork failed");
        odf::launch_group(g, plan->cfg[g], thr, bc, cs);
        if (cs != s && (hipEventRecord(plan->join[g], cs) != hipSuccess ||
                        hipStreamWaitEvent(s, plan->join[g], 0) != hipSuccess))
            return bfail(ODF_EHIP, "stream join failed");
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(ODF_EHIP, hipGetErrorString(e));
    return ODF_OK;
}

int odf_plan_info(const odf_plan* plan, int* njobs, long long* npix, int* ntiles, int* grids) {
    if (!plan) return ODF_EINVAL;
    if (njobs) *njobs = plan->njobs;
    if (npix) *npix = plan->npix;
    for (int c = 0; c < odf::kNumClasses; ++c) {
        if (ntiles) ntiles[c] = plan->class_tiles[c];
        if (grids) grids[c] = plan->class_tiles[c];  // one workgroup per tile
    }
    return ODF_OK;
}

int odf_plan_configs(const odf_plan* plan, int* configs) {
    if (!plan || !configs) return ODF_EINVAL;
    for (int g = 0; g < odf::kNumGroups; ++g) configs[g] = plan->cfg[g];
    return ODF_OK;
}

int odf_autotune_batch(int window, int kind, int reps, const char* cache_path, float* times_ms,
                       void* stream) {
    if (!odf::batch_window(window) || (kind != ODF_BVDF && kind != ODF_DDF) ||
        reps < 1)
        return odf::set_error(ODF_EINVAL, "autotune_batch: arguments out of range");
    const int grp = odf::batch_group(window, kind);
    // a mixed work list: frames and small images of several aspect ratios,
    // each with every pair term
    static const int kSizes[][2] = {{1080, 1920}, {720, 1280}, {512, 512}, {300, 400},
                                    {131, 97}, {64, 64}};
    constexpr int kImages = sizeof(kSizes) / sizeof(kSizes[0]);
    size_t off[kImages + 1] = {0};
    for (int i = 0; i < kImages; ++i) off[i + 1] = off[i] + (size_t)kSizes[i][0] * kSizes[i][1] * 3;
    std::vector<uint8_t> host;
    try {  // no exception crosses the C ABI
        host.resize(off[kImages]);
    } catch (...) {
        return odf::set_error(ODF_ENOMEM, "autotune_batch: host allocation failed");
    }
    for (int i = 0; i < kImages; ++i)
        odf::tuning_image(kSizes[i][0], kSizes[i][1], 2009 + i, host.data() + off[i]);
    uint8_t *img = nullptr, *out = nullptr;
    float ms[odf::kNumTileConfigs];
    int rc = ODF_OK, best = -1;
    std::vector<odf_job> jobs;
    if (odf::test_fail_alloc() || hipMalloc(&img, off[kImages]) != hipSuccess ||
        hipMalloc(&out, 3 * off[kImages]) != hipSuccess) {
        rc = odf::set_error(ODF_ENOMEM, "autotune_batch: device allocation failed");
        goto done;
    }
    if (hipMemcpy(img, host.data(), off[kImages], hipMemcpyHostToDevice) != hipSuccess) {
        rc = odf::set_error(ODF_EHIP, "autotune_batch: upload failed");
        goto done;
    }
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < kImages; ++i)
            jobs.push_back(odf_job{img + off[i], out + off[kImages] * d + off[i], nullptr,
                                   kSizes[i][0], kSizes[i][1], window, kind, d, 4, 0.25f});
    rc = time_group_shapes(jobs.data(), (int)jobs.size(), grp, reps, ms,
                           static_cast<hipStream_t>(stream));
    if (rc != ODF_OK) goto done;
    best = fastest(ms);
    odf::set_batch_tuned_config(grp, best);
    if (times_ms)
        for (int c = 0; c < odf::kNumTileConfigs; ++c) times_ms[c] = ms[c];
    rc = write_batch_line(cache_path, grp, best, ms);
done:
    if (img) (void)hipFree(img);
    if (out) (void)hipFree(out);
    return rc;
}

int odf_autotune_batch_jobs(const odf_job* jobs, int njobs, int reps, const char* cache_path,
                            float* times_ms, void* stream) {
    if (reps < 1) return odf::set_error(ODF_EINVAL, "autotune_batch_jobs: reps must be >= 1");
    if (odf::test_fail_alloc())
        return odf::set_error(ODF_ENOMEM, "autotune_batch_jobs: allocation failed");
    // validate every job once (a plan of the whole list, not launched)
    int cfg[odf::kNumGroups];
    for (int g = 0; g < odf::kNumGroups; ++g) cfg[g] = odf::batch_tuned_config(g);
    odf_plan* probe = nullptr;
    int rc = make_plan(jobs, njobs, cfg, &probe);
    if (rc != ODF_OK) return rc;
    destroy(probe);
    for (int g = 0; g < odf::kNumGroups; ++g) {
        float ms[odf::kNumTileConfigs];
        rc = time_group_shapes(jobs, njobs, g, reps, ms, static_cast<hipStream_t>(stream));
        if (rc != ODF_OK) return rc;
        if (times_ms)
            for (int c = 0; c < odf::kNumTileConfigs; ++c)
                times_ms[odf::kNumTileConfigs * g + c] = ms[c];
        const int best = fastest(ms);
        if (best < 0) continue;  // no job of this group
        odf::set_batch_tuned_config(g, best);
        rc = write_batch_line(cache_path, g, best, ms);
        if (rc != ODF_OK) return rc;
    }
    return ODF_OK;
}

int odf_plan_destroy(odf_plan* plan) {
    if (!plan) return ODF_EINVAL;
    destroy(plan);
    return ODF_OK;
}

}  // extern "C"
