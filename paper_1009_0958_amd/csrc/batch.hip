// batch.hip -- many uint8 images of different sizes, windows and filter
// variants in one persistent launch per kernel class.
//
// odf_batch_plan cuts every job into output tiles and uploads one work list
// per class (window, kind, pair term); each class kernel is persistent: its
// workgroups take tiles from the list with an atomic counter until it is
// exhausted.  One kernel per class keeps each class at the register budget of
// its own tile function (a single kernel branching over all of them would
// carry the largest budget, and spill, everywhere).  Tiles are ordered by
// decreasing size.  odf_batch_launch enqueues a counter
// reset kernel on the caller's stream, then the class kernels, forked onto
// per-plan auxiliary streams (default priority) and joined back with events
// so that classes run concurrently and their tails overlap; it allocates
// nothing and never synchronises, so it can be captured in a hipGraph.  Every tile writes
// only its own outputs with the same tile function as the per-image kernels,
// so results do not depend on which workgroup takes which tile.
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

// Filter tile t of a class work list (all fields are uniform over the
// workgroup and are moved to scalar registers).
template <int W, int KIND, int DIST, int SHAPE>
__device__ __forceinline__ void batch_tile(
    FwdSharedFor<W, KIND, DIST, true, BatchShape<SHAPE>::EXT_W, BatchShape<SHAPE>::EXT_H, false>& sh,
    const BatchClass& bc, int t) {
    constexpr int EXT_W = BatchShape<SHAPE>::EXT_W, EXT_H = BatchShape<SHAPE>::EXT_H;
    const BatchTile tile = bc.tiles[t];
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

template <int W>
constexpr int persistent_shape() {
    return W == 5 ? 1 : 0;
}

// Persistent form: workgroups take tiles with an atomic counter until the
// list is exhausted.
template <int W, int KIND, int DIST>
__global__ void __launch_bounds__(BatchShape<persistent_shape<W>()>::THREADS)
    batch_kernel(BatchClass bc) {
    constexpr int SHAPE = persistent_shape<W>();
    __shared__ FwdSharedFor<W, KIND, DIST, true, BatchShape<SHAPE>::EXT_W, BatchShape<SHAPE>::EXT_H, false> sh;
    __shared__ int s_tile;
    for (;;) {
        __syncthreads();  // the previous tile is finished with s_tile and sh
        if (threadIdx.x == 0) s_tile = atomicAdd(bc.counter, 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_tile);
        if (t >= bc.ntiles) break;
        batch_tile<W, KIND, DIST, SHAPE>(sh, bc, t);
    }
}

// Direct form: one workgroup per tile of the list, dispatched in list order.
template <int W, int KIND, int DIST, int SHAPE>
__global__ void __launch_bounds__(BatchShape<SHAPE>::THREADS)
    __attribute__((amdgpu_waves_per_eu(W == 3 && KIND != kACW ? 8 : 1))) batch_direct_kernel(BatchClass bc) {
    __shared__ FwdSharedFor<W, KIND, DIST, true, BatchShape<SHAPE>::EXT_W, BatchShape<SHAPE>::EXT_H, false> sh;
    batch_tile<W, KIND, DIST, SHAPE>(sh, bc, blockIdx.x);
}

__global__ void batch_reset(int* counters, int n) {
    if (threadIdx.x < n) counters[threadIdx.x] = 0;
}

// class = ((window == 5) * 2 + kind) * 3 + dist
static int class_window(int cls) { return cls / 6 ? 5 : 3; }

static void class_geometry(int cls, int shape, int& tw, int& th, int& threads) {
    const int h = class_window(cls) / 2;
    tw = BatchShape<0>::EXT_W - 2 * h;
    th = (shape == 0 ? BatchShape<0>::EXT_H : BatchShape<1>::EXT_H) - 2 * h;
    threads = shape == 0 ? BatchShape<0>::THREADS : BatchShape<1>::THREADS;
}

template <int W, int KIND>
static const void* persistent_kernel_wk(int dist) {
    if (dist == kExact) return reinterpret_cast<const void*>(&batch_kernel<W, KIND, kExact>);
    if (dist == kMinimax) return reinterpret_cast<const void*>(&batch_kernel<W, KIND, kMinimax>);
    return reinterpret_cast<const void*>(&batch_kernel<W, KIND, kRgb>);
}

static const void* persistent_kernel(int cls) {
    switch (cls / 3) {
    case 0: return persistent_kernel_wk<3, kBVDF>(cls % 3);
    case 1: return persistent_kernel_wk<3, kDDF>(cls % 3);
    case 2: return persistent_kernel_wk<5, kBVDF>(cls % 3);
    default: return persistent_kernel_wk<5, kDDF>(cls % 3);
    }
}

template <int W, int KIND, int DIST>
static void launch_class_wkd(bool direct, int shape, int grid, int threads, const BatchClass& bc,
                             hipStream_t s) {
    if (!direct)
        hipLaunchKernelGGL((batch_kernel<W, KIND, DIST>), dim3(grid), dim3(threads), 0, s, bc);
    else if (shape == 0)
        hipLaunchKernelGGL((batch_direct_kernel<W, KIND, DIST, 0>), dim3(bc.ntiles), dim3(threads),
                           0, s, bc);
    else
        hipLaunchKernelGGL((batch_direct_kernel<W, KIND, DIST, 1>), dim3(bc.ntiles), dim3(threads),
                           0, s, bc);
}

template <int W, int KIND>
static void launch_class_wk(int dist, bool direct, int shape, int grid, int threads,
                            const BatchClass& bc, hipStream_t s) {
    if (dist == kExact) launch_class_wkd<W, KIND, kExact>(direct, shape, grid, threads, bc, s);
    else if (dist == kMinimax) launch_class_wkd<W, KIND, kMinimax>(direct, shape, grid, threads, bc, s);
    else launch_class_wkd<W, KIND, kRgb>(direct, shape, grid, threads, bc, s);
}

static void launch_class(int cls, bool direct, int shape, int grid, int threads,
                         const BatchClass& bc, hipStream_t s) {
    switch (cls / 3) {
    case 0: launch_class_wk<3, kBVDF>(cls % 3, direct, shape, grid, threads, bc, s); break;
    case 1: launch_class_wk<3, kDDF>(cls % 3, direct, shape, grid, threads, bc, s); break;
    case 2: launch_class_wk<5, kBVDF>(cls % 3, direct, shape, grid, threads, bc, s); break;
    default: launch_class_wk<5, kDDF>(cls % 3, direct, shape, grid, threads, bc, s); break;
    }
}

}  // namespace odf

// Opaque plan (declared in odf.h).
struct odf_plan {
    odf::BatchJob* d_jobs = nullptr;
    odf::BatchTile* d_tiles = nullptr;
    int* d_counters = nullptr;
    int ntiles[odf::kNumClasses] = {};
    int offset[odf::kNumClasses] = {};
    int grid[odf::kNumClasses] = {};
    int shape[odf::kNumClasses] = {};
    int njobs = 0;
    long long npix = 0;
    int flags = 0;
    hipStream_t aux[odf::kNumClasses] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[odf::kNumClasses] = {};
};

namespace {

int bfail(int code, const char* msg) { return odf::set_error(code, "%s", msg); }


// Tile shape of a class: fixed for the persistent form, from the tuning
// table for the direct form.
int shape_of(int cls, int flags) {
    const int w = odf::class_window(cls);
    if (flags != ODF_BATCH_DIRECT) return w == 5 ? 1 : 0;
    const int cfg = odf::tuned_config(w, (cls / 3) % 2, cls % 3, true);
    int ew, eh;
    odf::tile_config_shape(cfg, &ew, &eh);
    return ew * eh >= 1024 ? 0 : 1;
}

void destroy(odf_plan* p) {
    if (!p) return;
    for (int c = 0; c < odf::kNumClasses; ++c) {
        if (p->aux[c]) (void)hipStreamDestroy(p->aux[c]);
        if (p->join[c]) (void)hipEventDestroy(p->join[c]);
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
    std::vector<std::pair<int, odf::BatchTile>> lists[odf::kNumClasses];
    long long npix = 0;
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
        const int cls = ((j.window == 5) * 2 + (j.kind == ODF_DDF)) * 3 + j.dist;
        int tw, th, thr;
        odf::class_geometry(cls, shape_of(cls, flags), tw, th, thr);
        for (int ty = 0; ty < j.M; ty += th)
            for (int tx = 0; tx < j.N; tx += tw) {
                // cost: output pixels of the (possibly clipped) tile
                const int cost = std::min(th, j.M - ty) * std::min(tw, j.N - tx);
                lists[cls].push_back({cost, odf::BatchTile{i, ty, tx}});
            }
        npix += (long long)j.M * j.N;
    }
    odf_plan* p = new (std::nothrow) odf_plan;
    if (!p) return bfail(ODF_ENOMEM, "plan allocation failed");
    std::vector<odf::BatchTile> all;
    for (int c = 0; c < odf::kNumClasses; ++c) {
        std::stable_sort(lists[c].begin(), lists[c].end(),
                         [](const std::pair<int, odf::BatchTile>& x,
                            const std::pair<int, odf::BatchTile>& y) { return x.first > y.first; });
        p->offset[c] = (int)all.size();
        p->ntiles[c] = (int)lists[c].size();
        for (auto& t : lists[c]) all.push_back(t.second);
    }
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
        destroy(p);
        return bfail(ODF_EHIP, "cannot query the compute unit count");
    }
    for (int c = 0; c < odf::kNumClasses; ++c) {
        int tw, th, thr, per_cu = 0;
        p->shape[c] = shape_of(c, flags);
        odf::class_geometry(c, p->shape[c], tw, th, thr);
        if (flags == ODF_BATCH_DIRECT) {
            p->grid[c] = p->ntiles[c];
            continue;
        }
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, odf::persistent_kernel(c), thr,
                                                         0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        p->grid[c] = std::min(p->ntiles[c], per_cu * cus);
    }
    if (hipMalloc(&p->d_jobs, sizeof(odf::BatchJob) * hj.size()) != hipSuccess ||
        hipMalloc(&p->d_tiles, sizeof(odf::BatchTile) * std::max<size_t>(1, all.size())) != hipSuccess ||
        hipMalloc(&p->d_counters, sizeof(int) * odf::kNumClasses) != hipSuccess) {
        destroy(p);
        return bfail(ODF_ENOMEM, "device allocation for the plan failed");
    }
    if (hipMemcpy(p->d_jobs, hj.data(), sizeof(odf::BatchJob) * hj.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(p->d_tiles, all.data(), sizeof(odf::BatchTile) * all.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(p->d_counters, 0, sizeof(int) * odf::kNumClasses) != hipSuccess) {
        destroy(p);
        return bfail(ODF_EHIP, "uploading the plan failed");
    }
    // auxiliary streams for every non-empty class after the first
    bool first = true;
    for (int c = 0; c < odf::kNumClasses; ++c) {
        if (p->ntiles[c] == 0) continue;
        if (first) { first = false; continue; }
        if (hipStreamCreateWithFlags(&p->aux[c], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->join[c], hipEventDisableTiming) != hipSuccess) {
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
    hipLaunchKernelGGL(odf::batch_reset, dim3(1), dim3(64), 0, s, plan->d_counters,
                       odf::kNumClasses);
    if (hipEventRecord(plan->fork, s) != hipSuccess) return bfail(ODF_EHIP, "fork event failed");
    for (int c = 0; c < odf::kNumClasses; ++c) {
        if (plan->ntiles[c] == 0) continue;
        odf::BatchClass bc{plan->d_jobs, plan->d_tiles + plan->offset[c], plan->d_counters + c,
                           plan->ntiles[c]};
        int tw, th, thr;
        odf::class_geometry(c, plan->shape[c], tw, th, thr);
        hipStream_t cs = plan->aux[c] ? plan->aux[c] : s;
        if (cs != s && hipStreamWaitEvent(cs, plan->fork, 0) != hipSuccess)
            return bfail(ODF_EHIP, "stream fork failed");
        odf::launch_class(c, plan->flags == ODF_BATCH_DIRECT, plan->shape[c], plan->grid[c], thr, bc,
                          cs);
        if (cs != s && (hipEventRecord(plan->join[c], cs) != hipSuccess ||
                        hipStreamWaitEvent(s, plan->join[c], 0) != hipSuccess))
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
        if (ntiles) ntiles[c] = plan->ntiles[c];
        if (grids) grids[c] = plan->grid[c];
    }
    return ODF_OK;
}

int odf_plan_destroy(odf_plan* plan) {
    if (!plan) return ODF_EINVAL;
    destroy(plan);
    return ODF_OK;
}

}  // extern "C"
