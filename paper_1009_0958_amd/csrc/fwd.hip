// fwd.hip -- forward kernel of the directional filters (BVDF / DDF) for gfx950.
//
// One workgroup owns an extended tile of EXT_H x EXT_W pixels (the output
// tile plus a halo of h = (w-1)/2 replicated-border pixels) and one thread
// per extended pixel.  For a member pixel p, its offset grid
// G_p(dy, dx) = theta(p, p + (dy, dx)), dy, dx in [-2h, 2h], holds every pair
// term any window containing p needs (Section II: the aggregate of member p
// in window c is the sum of G_p over the w x w box of W(c)).  Each unordered
// pixel pair is evaluated once (Sections 2.1-2.2 give the pair terms):
//
//   a1  load + prepare the pixel (direction, norms / chromaticity sums) -> LDS
//   a2  for each row group g = |dy| = 0..2h: compute the pair terms of
//       offsets (g, dx) (the "forward" half) for the own pixel, publish them
//       in an LDS plane, and read back the mirrored terms of row -g from the
//       pixels above (the pair (q, q + (g, -dx)) is row -g of p);
//       rows +g and -g are reduced at once into row sums of w consecutive
//       offsets;
//   a3  window aggregates = column sums of the row sums (w x w box sums of
//       G_p), one per window containing p; the summation tree is the same in
//       absolute pixel positions for every member of a window (rows left to
//       right, then rows top to bottom), so equal colours get bitwise-equal
//       aggregates and ties stay ties;
//   a4  objective (BVDF: A; DDF: A^(1-p) D^p compared as (1-p) log2 A + p log2 D)
//       and argmin by a 64-bit LDS atomicMin of (ordered objective, member
//       index): the smallest objective wins, ties go to the lowest index,
//       independent of the order of the atomics;
//       then the selected member is copied to the output.
#include "odf_internal.h"

namespace odf {

template <int W, int EXT_W, int EXT_H>
struct FwdGeom {
    static constexpr int H = W / 2;
    static constexpr int NW = W * W;
    static constexpr int G = 4 * H + 1;  // offsets per axis of a member's grid
    static constexpr int TW = EXT_W - 2 * H;
    static constexpr int TH = EXT_H - 2 * H;
    static constexpr int NT = EXT_W * EXT_H;
};

template <int W>
__device__ __forceinline__ void row_sums(const float (&row)[4 * (W / 2) + 1], float (&out)[W]) {
#pragma unroll
    for (int s = 0; s < W; ++s) {
        float acc = row[s];
#pragma unroll
        for (int k = 1; k < W; ++k) acc += row[s + k];
        out[s] = acc;
    }
}

// Aggregates of the own member p over every window containing it, for the
// angular term (L2PASS = false) or the L2 term of eq. (1) (L2PASS = true).
// agg[u] is the aggregate of p in the window c = p - offset(u).
template <int W, int KIND, int DIST, bool U8, int EXT_W, int EXT_H, bool L2PASS>
__device__ __forceinline__ void member_aggregates(const float4* __restrict__ s_dir,
                                                  const float4* __restrict__ s_raw,
                                                  float* __restrict__ s_plane, int ey, int ex,
                                                  int tid, const float4& mdir, const float4& mraw,
                                                  const MinimaxCoef& cf, float (&agg)[W * W]) {
    using Gm = FwdGeom<W, EXT_W, EXT_H>;
    constexpr int H = Gm::H, G = Gm::G, NT = Gm::NT;

    auto term = [&](int q) -> float {
        if (L2PASS) return l2_term(mraw, s_raw[q]);
        return pair_term<KIND, DIST, U8>(mdir, mraw, s_dir[q], s_raw[q], cf);
    };
    const float self =
        L2PASS ? 0.0f : pair_term<KIND, DIST, U8>(mdir, mraw, mdir, mraw, cf);

    float R[G][W];  // R[dy + 2h][s + 2h]: sum of G_p(dy, s .. s + w - 1)
#pragma unroll
    for (int g = 0; g <= 2 * H; ++g) {
        float own[G], up[G];
#pragma unroll
        for (int dx = -2 * H; dx <= 2 * H; ++dx) {
            own[dx + 2 * H] = 0.0f;
            if (g == 0 && dx <= 0) continue;
            const int py = ey + g, px = ex + dx;
            if (py < EXT_H && px >= 0 && px < EXT_W) {
                const float v = term(py * EXT_W + px);
                own[dx + 2 * H] = v;
                s_plane[(dx + 2 * H) * NT + tid] = v;
            }
        }
        __syncthreads();
#pragma unroll
        for (int dx = -2 * H; dx <= 2 * H; ++dx) {
            up[dx + 2 * H] = 0.0f;
            if (g == 0 && dx >= 0) continue;
            const int py = ey - g, px = ex + dx;
            if (py >= 0 && px >= 0 && px < EXT_W)
                up[dx + 2 * H] = s_plane[(2 * H - dx) * NT + py * EXT_W + px];
        }
        if (g == 0) {
            float row[G];
#pragma unroll
            for (int k = 0; k < G; ++k) row[k] = k < 2 * H ? up[k] : (k == 2 * H ? self : own[k]);
            row_sums<W>(row, R[2 * H]);
        } else {
            row_sums<W>(own, R[2 * H + g]);
            row_sums<W>(up, R[2 * H - g]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int uy = -H; uy <= H; ++uy) {
#pragma unroll
        for (int ux = -H; ux <= H; ++ux) {
            const int s = -H - ux + 2 * H;
            float acc = R[-H - uy + 2 * H][s];
#pragma unroll
            for (int dy = -H - uy + 1; dy <= H - uy; ++dy) acc += R[dy + 2 * H][s];
            agg[(uy + H) * W + (ux + H)] = acc;
        }
    }
}

template <int KIND>
__device__ __forceinline__ float objective_log(float A, float D, float p) {
    if (KIND == kBVDF || p == 0.0f) return A;
    if (p == 1.0f) return D;
    return fmaf(1.0f - p, __builtin_amdgcn_logf(A), p * __builtin_amdgcn_logf(D));
}

template <int KIND>
__device__ __forceinline__ float objective_value(float A, float D, float p) {
    if (KIND == kBVDF || p == 0.0f) return A;
    if (p == 1.0f) return D;
    return exp2f(fmaf(1.0f - p, log2f(A), p * log2f(D)));
}

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
