// fwd_launch.h -- the per-image forward kernel (one workgroup per output
// tile) and its launch templates; each window size is instantiated in a
// translation unit of its own (fwd.hip, fwd5.hip, fwd7.hip, fwd9.hip), and the
// strip form of each in another (fwd3s.hip .. fwd9s.hip), so that a parallel
// build compiles them side by side.
#pragma once

#include "fwd_strip.h"

namespace odf {

// Occupancy targets: 3x3 BVDF and DDF kernels are held to 64 VGPRs (8 waves
// per SIMD), the budget at which four 512-thread or two 1024-thread workgroups
// share a CU (ACWDDF keeps four objectives per window and cannot get there);
// 5x5 BVDF with the exact or rgb term to 80 (6 waves: three 512-thread
// workgroups), which it needs only a few registers more than; 7x7 BVDF to 128
// (4 waves instead of 3, for 84-240 B of spills: 11-16 % faster on uint8).
// Caps on 7x7 DDF, 5x5 ACWDDF and 5x5 BVDF minimax measured 4-8 % slower.
template <int W, int KIND, int DIST>
constexpr int fwd_waves_per_eu() {
    if (W == 3 && !centre_weighted(KIND)) return 8;
    if (W == 5 && KIND == kBVDF && DIST != kMinimax) return 6;
    if (W == 7 && KIND == kBVDF) return 4;
    return 1;
}

template <int W, int KIND, int DIST, bool U8, int EXT_W, int EXT_H, bool AGG>
__global__ void __launch_bounds__(EXT_W* EXT_H)
    __attribute__((amdgpu_waves_per_eu(AGG ? 1 : fwd_waves_per_eu<W, KIND, DIST>())))
    fwd_kernel(FwdParams prm) {
    __shared__ FwdSharedFor<W, KIND, DIST, U8, EXT_W, EXT_H, AGG> sh;
    using Gm = FwdGeom<W, EXT_W, EXT_H>;
    const int t = flat_block(prm.grid.n);
    if (t < 0) return;
    const TileCoord c = tile_coord(t, prm.grid);
    fwd_tile<W, KIND, DIST, U8, EXT_W, EXT_H, AGG>(sh, prm, c.b, c.ty * Gm::TH, c.tx * Gm::TW,
                                                   threadIdx.x);
}

template <int W, int KIND, int DIST, bool U8, bool AGG, int EXT_W, int EXT_H>
static hipError_t launch_shape(const FwdParams& prm, hipStream_t stream) {
    using Gm = FwdGeom<W, EXT_W, EXT_H>;
    FwdParams q = prm;
    q.grid = tile_grid(prm.B, (prm.N + Gm::TW - 1) / Gm::TW, (prm.M + Gm::TH - 1) / Gm::TH);
    hipLaunchKernelGGL((fwd_kernel<W, KIND, DIST, U8, EXT_W, EXT_H, AGG>), flat_grid(q.grid.n),
                       dim3(Gm::NT), 0, stream, q);
    return hipGetLastError();
}

template <int W, int KIND, int DIST, bool U8, bool AGG>
static hipError_t launch_t(int cfg, const FwdParams& prm, hipStream_t stream) {
    if constexpr (AGG) {  // inspection path: one shape (it keeps every aggregate live)
        (void)cfg;
        return launch_shape<W, KIND, DIST, U8, AGG, 32, 16>(prm, stream);
    } else if constexpr (W == 9) {  // 512 threads, 8 output rows: the one tile shape offered
        if (cfg == 2) return launch_shape<W, KIND, DIST, U8, AGG, 32, 16>(prm, stream);
        if constexpr (strip_form<W, KIND, U8>())
            if (is_strip_config(cfg))
                return launch_strip_extern<W>(KIND, DIST, U8, prm, strip_bands(cfg), stream);
        return hipErrorInvalidValue;
    } else if constexpr ((W == 5 && centre_weighted(KIND)) || W == 7) {
        switch (cfg) {
        case 2: return launch_shape<W, KIND, DIST, U8, AGG, 32, 16>(prm, stream);
        case 3: return launch_shape<W, KIND, DIST, U8, AGG, 64, 8>(prm, stream);
        default:
            if constexpr (strip_form<W, KIND, U8>())
                if (is_strip_config(cfg))
                    return launch_strip_extern<W>(KIND, DIST, U8, prm, strip_bands(cfg), stream);
            return hipErrorInvalidValue;
        }
    } else {
        switch (cfg) {
        case 0: return launch_shape<W, KIND, DIST, U8, AGG, 32, 32>(prm, stream);
        case 1: return launch_shape<W, KIND, DIST, U8, AGG, 64, 16>(prm, stream);
        case 2: return launch_shape<W, KIND, DIST, U8, AGG, 32, 16>(prm, stream);
        case 3: return launch_shape<W, KIND, DIST, U8, AGG, 64, 8>(prm, stream);
        default:
            if constexpr (strip_form<W, KIND, U8>())  // 32-wide strips of 8 or 3 bands of 16 rows
                if (is_strip_config(cfg))
                    return launch_strip_extern<W>(KIND, DIST, U8, prm, strip_bands(cfg), stream);
            return hipErrorInvalidValue;
        }
    }
}

template <int W, int KIND, int DIST>
static hipError_t launch_wkd(bool u8, bool agg, int cfg, const FwdParams& prm, hipStream_t s) {
    if constexpr (centre_weighted(KIND)) {  // no aggregate-inspection form
        if (agg) return hipErrorInvalidValue;
        return u8 ? launch_t<W, KIND, DIST, true, false>(cfg, prm, s)
                  : launch_t<W, KIND, DIST, false, false>(cfg, prm, s);
    } else {
        if (u8) return agg ? launch_t<W, KIND, DIST, true, true>(cfg, prm, s)
                           : launch_t<W, KIND, DIST, true, false>(cfg, prm, s);
        return agg ? launch_t<W, KIND, DIST, false, true>(cfg, prm, s)
                   : launch_t<W, KIND, DIST, false, false>(cfg, prm, s);
    }
}

template <int W, int KIND>
static hipError_t launch_wk(int dist, bool u8, bool agg, int cfg, const FwdParams& prm,
                            hipStream_t s) {
    if constexpr (KIND == kCWV) return launch_wkd<W, KIND, kRgb>(u8, agg, cfg, prm, s);  // no angle
    switch (dist) {
    case kExact: return launch_wkd<W, KIND, kExact>(u8, agg, cfg, prm, s);
    case kMinimax: return launch_wkd<W, KIND, kMinimax>(u8, agg, cfg, prm, s);
    default: return launch_wkd<W, KIND, kRgb>(u8, agg, cfg, prm, s);
    }
}

template <int W>
static hipError_t launch_w(int kind, int dist, bool u8, bool agg, int cfg, const FwdParams& prm,
                           hipStream_t s) {
    if (kind == kBVDF) return launch_wk<W, kBVDF>(dist, u8, agg, cfg, prm, s);
    if (kind == kDDF) return launch_wk<W, kDDF>(dist, u8, agg, cfg, prm, s);
    if constexpr (W >= 9) return hipErrorInvalidValue;  // no 9x9 centre-weighted filters
    else if (kind == kACW) return launch_wk<W, kACW>(dist, u8, agg, cfg, prm, s);
    else if (kind == kCW) return launch_wk<W, kCW>(dist, u8, agg, cfg, prm, s);
    else return launch_wk<W, kCWV>(dist, u8, agg, cfg, prm, s);
}

// Launchers of the window sizes instantiated in fwd5.hip, fwd7.hip and fwd9.hip.
hipError_t launch_forward5(int kind, int dist, bool u8, bool aggregates, int cfg,
                           const FwdParams& prm, hipStream_t stream);
hipError_t launch_forward7(int kind, int dist, bool u8, bool aggregates, int cfg,
                           const FwdParams& prm, hipStream_t stream);
hipError_t launch_forward9(int kind, int dist, bool u8, bool aggregates, int cfg,
                           const FwdParams& prm, hipStream_t stream);

}  // namespace odf
