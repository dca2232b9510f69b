// fwd.hip -- forward kernel of the directional filters (BVDF / DDF) for gfx950.
//
// Per workgroup tile (see aggregates.h for a2/a3):
//   a1  load + prepare the pixel (direction, norms / chromaticity sums) -> LDS
//   a2  pair terms, each unordered pixel pair once, via LDS row-group planes
//   a3  canonical-order box sums -> aggregates of every (member, window)
//   a4  objective (BVDF: A; DDF: A^(1-p) D^p compared as (1-p) log2 A + p log2 D)
//       and argmin by a 64-bit LDS atomicMin of (ordered objective, member
//       index): the smallest objective wins, ties go to the lowest index,
//       independent of the order of the atomics; then the selected member is
//       copied to the output.
#include "aggregates.h"
#include "odf_internal.h"

namespace odf {

template <int W, int KIND, int DIST, bool U8, int EXT_W, int EXT_H, bool AGG>
__global__ void __launch_bounds__(EXT_W* EXT_H) fwd_kernel(FwdParams prm) {
    using Gm = FwdGeom<W, EXT_W, EXT_H>;
    constexpr int H = Gm::H, NW = Gm::NW, G = Gm::G, TW = Gm::TW, TH = Gm::TH, NT = Gm::NT;

    __shared__ float4 s_dir[NT];
    __shared__ float4 s_raw[NT];
    __shared__ float s_plane[G * NT];
    __shared__ unsigned long long s_key[AGG ? 1 : TH * TW];

    const int tid = threadIdx.x;
    const int ey = tid / EXT_W, ex = tid - ey * EXT_W;
    const int b = blockIdx.z;
    const int ty0 = blockIdx.y * TH, tx0 = blockIdx.x * TW;
    const int M = prm.M, N = prm.N;

    // a1: own extended pixel, replicated border
    {
        const int gy = min(max(ty0 - H + ey, 0), M - 1);
        const int gx = min(max(tx0 - H + ex, 0), N - 1);
        const size_t pix = ((size_t)b * M + gy) * N + gx;
        float x0, x1, x2;
        if (U8) {
            const uint8_t* s = static_cast<const uint8_t*>(prm.img) + pix * 3;
            x0 = s[0]; x1 = s[1]; x2 = s[2];
        } else {
            const float* s = static_cast<const float*>(prm.img) + pix * 3;
            x0 = s[0]; x1 = s[1]; x2 = s[2];
        }
        float4 d, r;
        prepare_pixel<DIST, U8>(x0, x1, x2, d, r);
        s_dir[tid] = d;
        s_raw[tid] = r;
    }
    if (!AGG)
        for (int i = tid; i < TH * TW; i += NT) s_key[i] = ~0ull;
    __syncthreads();
    const float4 mdir = s_dir[tid];
    const float4 mraw = s_raw[tid];

    // a2 + a3
    float A[NW], D[NW];
    member_aggregates<W, KIND, DIST, U8, EXT_W, EXT_H, false>(s_dir, s_raw, s_plane, ey, ex, tid,
                                                             mdir, mraw, prm.coef, A);
    if (KIND == kDDF)
        member_aggregates<W, KIND, DIST, U8, EXT_W, EXT_H, true>(s_dir, s_raw, s_plane, ey, ex,
                                                                tid, mdir, mraw, prm.coef, D);
    else
#pragma unroll
        for (int u = 0; u < NW; ++u) D[u] = 0.0f;

    // a4: objective of this member in every window of the tile containing it
#pragma unroll
    for (int u = 0; u < NW; ++u) {
        const int cy = ey - u / W;  // window centre, tile-local
        const int cx = ex - u % W;
        if (cy < 0 || cy >= TH || cx < 0 || cx >= TW) continue;
        if (ty0 + cy >= M || tx0 + cx >= N) continue;
        if (AGG) {
            const size_t o = (((size_t)b * M + ty0 + cy) * N + tx0 + cx) * NW + u;
            prm.dbg_A[o] = A[u];
            if (prm.dbg_D) prm.dbg_D[o] = D[u];
            if (prm.dbg_O) prm.dbg_O[o] = objective_value<KIND>(A[u], D[u], prm.p);
        } else {
            const float om = objective_log<KIND>(A[u], D[u], prm.p);
            const unsigned long long key = ((unsigned long long)order_key(om) << 32) | (unsigned)u;
            atomicMin(&s_key[cy * TW + cx], key);
        }
    }
    if (AGG) return;
    __syncthreads();

    // write the selected member of every window of the tile
    for (int i = tid; i < TH * TW; i += NT) {
        const int cy = i / TW, cx = i - (i / TW) * TW;
        const int gy = ty0 + cy, gx = tx0 + cx;
        if (gy >= M || gx >= N) continue;
        const int u = min((int)(s_key[i] & 0xffu), NW - 1);
        const float4 r = s_raw[(cy + u / W) * EXT_W + cx + u % W];
        const size_t pix = ((size_t)b * M + gy) * N + gx;
        if (U8) {
            uint8_t* o = static_cast<uint8_t*>(prm.out) + pix * 3;
            o[0] = (uint8_t)r.x; o[1] = (uint8_t)r.y; o[2] = (uint8_t)r.z;
        } else {
            float* o = static_cast<float*>(prm.out) + pix * 3;
            o[0] = r.x; o[1] = r.y; o[2] = r.z;
        }
        if (prm.idx) prm.idx[pix] = (uint8_t)u;
    }
}

template <int W, int KIND, int DIST, bool U8, bool AGG>
static hipError_t launch_t(const FwdParams& prm, hipStream_t stream) {
    // 5x5 DDF keeps both aggregates live: half-size tiles leave it more registers
    constexpr int EXT_W = 32, EXT_H = (W == 5 && KIND == kDDF) ? 16 : 32;
    using Gm = FwdGeom<W, EXT_W, EXT_H>;
    dim3 grid((prm.N + Gm::TW - 1) / Gm::TW, (prm.M + Gm::TH - 1) / Gm::TH, prm.B);
    hipLaunchKernelGGL((fwd_kernel<W, KIND, DIST, U8, EXT_W, EXT_H, AGG>), grid, dim3(Gm::NT), 0,
                       stream, prm);
    return hipGetLastError();
}

template <int W, int KIND, int DIST>
static hipError_t launch_wkd(bool u8, bool agg, const FwdParams& prm, hipStream_t s) {
    if (u8) return agg ? launch_t<W, KIND, DIST, true, true>(prm, s)
                       : launch_t<W, KIND, DIST, true, false>(prm, s);
    return agg ? launch_t<W, KIND, DIST, false, true>(prm, s)
               : launch_t<W, KIND, DIST, false, false>(prm, s);
}

template <int W, int KIND>
static hipError_t launch_wk(int dist, bool u8, bool agg, const FwdParams& prm, hipStream_t s) {
    switch (dist) {
    case kExact: return launch_wkd<W, KIND, kExact>(u8, agg, prm, s);
    case kMinimax: return launch_wkd<W, KIND, kMinimax>(u8, agg, prm, s);
    default: return launch_wkd<W, KIND, kRgb>(u8, agg, prm, s);
    }
}

template <int W>
static hipError_t launch_w(int kind, int dist, bool u8, bool agg, const FwdParams& prm,
                           hipStream_t s) {
    return kind == kBVDF ? launch_wk<W, kBVDF>(dist, u8, agg, prm, s)
                         : launch_wk<W, kDDF>(dist, u8, agg, prm, s);
}

hipError_t launch_forward(int window, int kind, int dist, bool u8, bool aggregates,
                          const FwdParams& prm, hipStream_t stream) {
    if (window == 3) return launch_w<3>(kind, dist, u8, aggregates, prm, stream);
    return launch_w<5>(kind, dist, u8, aggregates, prm, stream);
}

}  // namespace odf
