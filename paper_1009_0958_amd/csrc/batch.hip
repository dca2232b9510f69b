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
// budget everywhere), so they keep kernels of their own.  odf_batch_launch
// enqueues (persistent form) a counter reset kernel on the caller's stream,
// then the group kernels, forked onto per-plan auxiliary streams (default priority) and
// joined back with events so that groups run concurrently and their tails
// overlap; it allocates nothing and never synchronises, so it can be captured
// in a hipGraph.  Every tile writes only its own outputs with the same tile
// function as the per-image kernels, so results do not depend on which
// workgroup takes which tile.
#include <algorithm>
#include <new>
#include <vector>

#include "fwd_tile.h"
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
    int* counter;
    int ntiles;
};

// Extended-tile shapes of the batch kernels: 0 = 32 x 32, 1 = 32 x 16.  The
// persistent form uses 32 x 32 for 3x3 and 32 x 16 for 5x5 (its loop needs
// more registers than a 1024-thread 5x5 tile allows); the direct form takes
// the shape the tuning table holds for the class (1024-thread entries map to
// 32 x 32, 512-thread ones to 32 x 16).
template <int SHAPE>
struct BatchShape {
    static constexpr int EXT_W = 32;
    static constexpr int EXT_H = SHAPE == 0 ? 32 : 16;
    static constexpr int THREADS = EXT_W * EXT_H;
};

constexpr int kNumClasses = 12;  // (window 3/5) x (BVDF/DDF) x (exact/minimax/rgb)

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
template <int W, int KIND, int DIST, int SHAPE>
__device__ __forceinline__ void batch_tile(
    FwdSharedFor<W, KIND, DIST, true, BatchShape<SHAPE>::EXT_W, BatchShape<SHAPE>::EXT_H, false>& sh,
    const BatchClass& bc, const BatchTile& tile) {
    constexpr int EXT_W = BatchShape<SHAPE>::EXT_W, EXT_H = BatchShape<SHAPE>::EXT_H;
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
    // an opaque copy of the thread index keeps the tile's address arithmetic
    // inside a persistent loop instead of hoisted and held in registers
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    fwd_tile<W, KIND, DIST, true, EXT_W, EXT_H, false>(sh, prm, 0, uni(tile.ty0), uni(tile.tx0), tid);
}

// LDS of a group kernel: room for the tile of any pair term.
template <int W, int KIND, int SHAPE>
struct BatchSmem {
    template <int DIST>
    using Sh = FwdSharedFor<W, KIND, DIST, true, BatchShape<SHAPE>::EXT_W,
                            BatchShape<SHAPE>::EXT_H, false>;
    static constexpr size_t a = sizeof(Sh<kExact>), b = sizeof(Sh<kMinimax>),
                            c = sizeof(Sh<kRgb>);
    static constexpr size_t BYTES = a > b ? (a > c ? a : c) : (b > c ? b : c);
};

// Tile t of a group list: its pair term comes from the job (uniform branch).
template <int W, int KIND, int SHAPE>
__device__ __forceinline__ void batch_tile_any(char* smem, const BatchClass& bc, int t) {
    const BatchTile tile = bc.tiles[t];
    const int dist = uni(bc.jobs[uni(tile.job)].dist);
    using S = BatchSmem<W, KIND, SHAPE>;
    if (dist == kExact)
        batch_tile<W, KIND, kExact, SHAPE>(*reinterpret_cast<typename S::template Sh<kExact>*>(smem),
                                           bc, tile);
    else if (dist == kMinimax)
        batch_tile<W, KIND, kMinimax, SHAPE>(
            *reinterpret_cast<typename S::template Sh<kMinimax>*>(smem), bc, tile);
    else
        batch_tile<W, KIND, kRgb, SHAPE>(*reinterpret_cast<typename S::template Sh<kRgb>*>(smem),
                                         bc, tile);
}

template <int W>
constexpr int persistent_shape() {
    return W == 5 ? 1 : 0;
}

// Persistent form: workgroups take tiles with an atomic counter until the
// list is exhausted.
template <int W, int KIND>
__global__ void __launch_bounds__(BatchShape<persistent_shape<W>()>::THREADS)
    batch_kernel(BatchClass bc) {
    constexpr int SHAPE = persistent_shape<W>();
    __shared__ __align__(16) char smem[BatchSmem<W, KIND, SHAPE>::BYTES];
    __shared__ int s_tile;
    for (;;) {
        __syncthreads();  // the previous tile is finished with s_tile and smem
        if (threadIdx.x == 0) s_tile = atomicAdd(bc.counter, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_tile);
        if (t >= bc.ntiles) break;
        batch_tile_any<W, KIND, SHAPE>(smem, bc, t);
    }
}

// Direct form: one workgroup per tile of the list, dispatched in list order.
template <int W, int KIND, int SHAPE>
__global__ void __launch_bounds__(BatchShape<SHAPE>::THREADS)
    __attribute__((amdgpu_waves_per_eu(W == 3 && KIND != kACW ? 8 : 1))) batch_direct_kernel(BatchClass bc) {
    __shared__ __align__(16) char smem[BatchSmem<W, KIND, SHAPE>::BYTES];
    const int t = flat_block(bc.ntiles);
    if (t < 0) return;
    batch_tile_any<W, KIND, SHAPE>(smem, bc, t);
}

__global__ void batch_reset(int* counters, int n) {
    if (threadIdx.x < n) counters[threadIdx.x] = 0;
}

// class = ((window == 5) * 2 + kind) * 3 + dist; group = class / 3
constexpr int kNumGroups = kNumClasses / 3;
static int group_window(int grp) { return grp / 2 ? 5 : 3; }

static void group_geometry(int grp, int shape, int& tw, int& th, int& threads) {
    const int h = group_window(grp) / 2;
    tw = BatchShape<0>::EXT_W - 2 * h;
    th = (shape == 0 ? BatchShape<0>::EXT_H : BatchShape<1>::EXT_H) - 2 * h;
    threads = shape == 0 ? BatchShape<0>::THREADS : BatchShape<1>::THREADS;
}

static const void* persistent_kernel(int grp) {
    switch (grp) {
    case 0: return reinterpret_cast<const void*>(&batch_kernel<3, kBVDF>);
    case 1: return reinterpret_cast<const void*>(&batch_kernel<3, kDDF>);
    case 2: return reinterpret_cast<const void*>(&batch_kernel<5, kBVDF>);
    default: return reinterpret_cast<const void*>(&batch_kernel<5, kDDF>);
    }
}

template <int W, int KIND>
static void launch_group_wk(bool direct, int shape, int grid, int threads, const BatchClass& bc,
                            hipStream_t s) {
    if (!direct)
        hipLaunchKernelGGL((batch_kernel<W, KIND>), dim3(grid), dim3(threads), 0, s, bc);
    else if (shape == 0)
        hipLaunchKernelGGL((batch_direct_kernel<W, KIND, 0>), flat_grid(bc.ntiles), dim3(threads),
                           0, s, bc);
    else
        hipLaunchKernelGGL((batch_direct_kernel<W, KIND, 1>), flat_grid(bc.ntiles), dim3(threads),
                           0, s, bc);
}

static void launch_group(int grp, bool direct, int shape, int grid, int threads,
                         const BatchClass& bc, hipStream_t s) {
    switch (grp) {
    case 0: launch_group_wk<3, kBVDF>(direct, shape, grid, threads, bc, s); break;
    case 1: launch_group_wk<3, kDDF>(direct, shape, grid, threads, bc, s); break;
    case 2: launch_group_wk<5, kBVDF>(direct, shape, grid, threads, bc, s); break;
    default: launch_group_wk<5, kDDF>(direct, shape, grid, threads, bc, s); break;
    }
}

}  // namespace odf

// Opaque plan (declared in odf.h).
struct odf_plan {
    odf::BatchJob* d_jobs = nullptr;
    odf::BatchTile* d_tiles = nullptr;
    int* d_counters = nullptr;
    int class_tiles[odf::kNumClasses] = {};  // per class, for odf_plan_info
    int ntiles[odf::kNumGroups] = {};
    int offset[odf::kNumGroups] = {};
    int grid[odf::kNumGroups] = {};
    int shape[odf::kNumGroups] = {};
    int njobs = 0;
    long long npix = 0;
    int flags = 0;
    hipStream_t aux[odf::kNumGroups] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[odf::kNumGroups] = {};
};

namespace {

int bfail(int code, const char* msg) { return odf::set_error(code, "%s", msg); }

// Tile shape of a group.  A plan is one launch over many tiles, so the shape
// with the best steady-state rate wins (measured on MI355X on 3840 x 2160
// frames: 32 x 32 for 3x3 DDF, 32 x 16 for 3x3 BVDF and for 5x5); the
// per-image tuning table, chosen where a single image's last partial wave of
// workgroups matters, is not consulted.  The persistent form's loop needs
// 32 x 16 for 5x5 (registers).
int shape_of(int grp, int flags) {
    const int w = odf::group_window(grp);
    if (flags != ODF_BATCH_DIRECT) return w == 5 ? 1 : 0;
    return (w == 3 && grp % 2 == ODF_DDF) ? 0 : 1;
}

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
    (void)hipFree(p->d_counters);
    delete p;
}

}  // namespace

extern "C" {

int odf_batch_plan(const odf_job* jobs, int njobs, odf_plan** plan, void* stream) {
    return odf_batch_plan_ex(jobs, njobs, ODF_BATCH_DIRECT, plan, stream);
}

int odf_batch_plan_ex(const odf_job* jobs, int njobs, int flags, odf_plan** plan, void* stream) {
    (void)stream;
    if (flags != ODF_BATCH_PERSISTENT && flags != ODF_BATCH_DIRECT)
        return bfail(ODF_EINVAL, "flags must be ODF_BATCH_PERSISTENT or ODF_BATCH_DIRECT");
    if (!plan) return bfail(ODF_EINVAL, "plan is NULL");
    *plan = nullptr;
    if (!jobs || njobs < 1) return bfail(ODF_EINVAL, "jobs must be a non-empty array");
    std::vector<odf::BatchJob> hj(njobs);
    for (int i = 0; i < njobs; ++i) {
        const odf_job& j = jobs[i];
        if (!j.img || !j.out) return bfail(ODF_EINVAL, "job img/out is NULL");
        if (j.M < 1 || j.N < 1 || (long long)j.M * j.N >= (1ll << 31))
            return bfail(ODF_EINVAL, "job size out of range");
        if (j.window != 3 && j.window != 5) return bfail(ODF_EUNSUPPORTED, "job window not 3 or 5");
        if (j.kind != ODF_BVDF && j.kind != ODF_DDF) return bfail(ODF_EINVAL, "job kind out of range");
        if (j.dist < ODF_EXACT || j.dist > ODF_RGB) return bfail(ODF_EINVAL, "job dist out of range");
        if (j.dist == ODF_MINIMAX && (j.q < 2 || j.q > 4)) return bfail(ODF_EINVAL, "job q out of range");
        if (j.kind == ODF_DDF && !(j.p >= 0.0f && j.p <= 1.0f)) return bfail(ODF_EINVAL, "job p out of range");
        const size_t nb = (size_t)j.M * j.N * 3;
        const char* a = (const char*)j.img;
        const char* o = (const char*)j.out;
        if (a < o + nb && o < a + nb) return bfail(ODF_EINVAL, "job out overlaps img");
    }
    int shape[odf::kNumGroups];
    for (int g = 0; g < odf::kNumGroups; ++g) shape[g] = shape_of(g, flags);

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
        const int grp = (j.window == 5) * 2 + (j.kind == ODF_DDF);
        int tw, th, thr;
        odf::group_geometry(grp, shape[grp], tw, th, thr);
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
        for (auto& t : lists[g]) all.push_back(t.second);
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
        destroy(p);
        return bfail(ODF_EHIP, "cannot query the compute unit count");
    }
    for (int g = 0; g < odf::kNumGroups; ++g) {
        int tw, th, thr, per_cu = 0;
        p->shape[g] = shape[g];
        odf::group_geometry(g, p->shape[g], tw, th, thr);
        if (flags == ODF_BATCH_DIRECT) {
            p->grid[g] = p->ntiles[g];
            continue;
        }
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, odf::persistent_kernel(g), thr,
                                                         0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        p->grid[g] = std::min(p->ntiles[g], per_cu * cus);
    }
    if (hipMalloc(&p->d_jobs, sizeof(odf::BatchJob) * hj.size()) != hipSuccess ||
        hipMalloc(&p->d_tiles, sizeof(odf::BatchTile) * std::max<size_t>(1, all.size())) != hipSuccess ||
        hipMalloc(&p->d_counters, sizeof(int) * odf::kNumGroups) != hipSuccess) {
        destroy(p);
        return bfail(ODF_ENOMEM, "device allocation for the plan failed");
    }
    if (hipMemcpy(p->d_jobs, hj.data(), sizeof(odf::BatchJob) * hj.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->d_tiles, all.data(), sizeof(odf::BatchTile) * all.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(p->d_counters, 0, sizeof(int) * odf::kNumGroups) != hipSuccess) {
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
    p->flags = flags;
    *plan = p;
    return ODF_OK;
}

int odf_batch_launch(const odf_plan* plan, void* stream) {
    if (!plan) return bfail(ODF_EINVAL, "plan is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool direct = plan->flags == ODF_BATCH_DIRECT;
    if (!direct)  // the persistent kernels' tile counters start at 0
        hipLaunchKernelGGL(odf::batch_reset, dim3(1), dim3(64), 0, s, plan->d_counters,
                           odf::kNumGroups);
    if (hipEventRecord(plan->fork, s) != hipSuccess) return bfail(ODF_EHIP, "fork event failed");
    for (int g = 0; g < odf::kNumGroups; ++g) {
        if (plan->ntiles[g] == 0) continue;
        odf::BatchClass bc{plan->d_jobs, plan->d_tiles + plan->offset[g], plan->d_counters + g,
                           plan->ntiles[g]};
        int tw, th, thr;
        odf::group_geometry(g, plan->shape[g], tw, th, thr);
        hipStream_t cs = plan->aux[g] ? plan->aux[g] : s;
        if (cs != s && hipStreamWaitEvent(cs, plan->fork, 0) != hipSuccess)
            return bfail(ODF_EHIP, "stream fork failed");
        odf::launch_group(g, direct, plan->shape[g], plan->grid[g], thr, bc, cs);
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
        const int g = c / 3;
        if (ntiles) ntiles[c] = plan->class_tiles[c];
        // workgroups launched for the class's tiles: one per tile (direct) or
        // the grid of its group's persistent kernel
        if (grids)
            grids[c] = plan->class_tiles[c] == 0 ? 0
                       : (plan->flags == ODF_BATCH_DIRECT ? plan->class_tiles[c] : plan->grid[g]);
    }
    return ODF_OK;
}

int odf_plan_destroy(odf_plan* plan) {
    if (!plan) return ODF_EINVAL;
    destroy(plan);
    return ODF_OK;
}

}  // extern "C"
