// aggregates.h -- per-member window aggregates over a workgroup tile (shared
// by the forward filter and the softmin kernels).
//
// One workgroup owns an extended tile of EXT_H x EXT_W pixels (the output
// tile plus a halo of h = (w-1)/2 pixels) with one thread per extended
// pixel.  For a member pixel p, its offset grid
// G_p(dy, dx) = theta(p, p + (dy, dx)), dy, dx in [-2h, 2h], holds every pair
// term a window containing p needs: the aggregate of p in window c is the sum
// of G_p over the w x w box of W(c) (Section II, eqs. 2-3).  Each unordered
// pixel pair is evaluated once: for each row group g = |dy| = 0..2h the
// thread computes the pair terms of offsets (g, dx) of its own pixel,
// publishes them in an LDS plane, and reads back the mirrored terms of row -g
// from the pixels above.  Rows +g and -g are reduced at once into row sums of
// w consecutive offsets; the window aggregates are the column sums of those
// row sums.  The summation tree is the same in absolute pixel positions for
// every member of a window (rows left to right, then rows top to bottom), so
// equal colours get bitwise-equal aggregates and ties stay ties.
#pragma once

#include <type_traits>

#include "pair_terms.h"

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

// The box sums are plain additions: contraction is off, so a pair term whose last
// operation is a multiply (the BVDF chromaticity distance) is never fused into the
// sum where the thread computed it but left unfused where it was read from LDS --
// that would round the same term two ways and break the exact ties of equal colours.
template <int W>
__device__ __forceinline__ void row_sums(const float (&row)[4 * (W / 2) + 1], float (&out)[W]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int s = 0; s < W; ++s) {
        float acc = row[s];
#pragma unroll
        for (int k = 1; k < W; ++k) acc += row[s + k];
        out[s] = acc;
    }
}

// LDS view of a tile's prepared pixels (pair_terms.h): float inputs use dir
// and raw, uint8 inputs dir and, for MINIMAX and RGB, the aux2 plane inv.
struct TilePix {
    const float4* dir;
    const float4* raw;
    const float* inv;
};

// Makes each value exist at this point of the program (an empty asm that
// takes them as operands): the compiler may not sink their computation past it.
template <int K>
__device__ __forceinline__ void pin_values(const float (&v)[K]) {
#pragma unroll
    for (int i = 0; i < K; ++i) asm volatile("" ::"v"(v[i]));
}

// The default plane hook of member_aggregates_x: nothing.
struct NoPlaneHook {
    __device__ __forceinline__ void before(int) const {}
    __device__ __forceinline__ void after(int) const {}
};

// Aggregates of the own member p over every window containing it.  PASS 0:
// the angular term into agg0; PASS 1: the L2 term of eq. (1) into agg0;
// PASS 2: both in one sweep (angular -> agg0, L2 -> agg1) with two LDS plane
// sets, sharing the neighbour loads, bounds tests and barriers.  agg[u] is the
// aggregate of p in the window c = p - offset(u).  CEN: also cen[u] = the term
// of p and that window's centre c (taken from the offset grid, so no extra
// pair is evaluated).  s_plane holds G * NT floats per term.  mraw.w is the
// member's aux2 (uint8 layout: its other fields are unused).
//
// GUARD = false drops the tests that keep neighbours inside the extended tile:
// a neighbour index then runs past the pixel arrays by up to 2h rows + 2h and a
// mirrored read before the plane by as much, into whatever LDS the caller
// placed there (it must be part of the same allocation).  The pair terms so
// formed are meaningless, but they only enter row sums of windows that reach
// outside the extended tile -- every window of the output tile has all its
// members inside it -- so the caller must discard the objectives of those
// windows.
//
// PSTRIDE (0: NT) is the distance between two planes; HOOK is called in every
// row group g with the sweep's own terms written (before(g), ahead of the
// barrier that publishes them) and published (after(g), ahead of the barrier
// that ends the group): the strip kernels use it to carry the planes of a
// band's last rows into the next band.
template <int W, int KIND, int DIST, bool U8, int EXT_W, int EXT_H, int PASS, bool CEN,
          bool GUARD, int PSTRIDE = 0, class HOOK = NoPlaneHook>
__device__ __forceinline__ void member_aggregates_x(
    const TilePix& px, float* __restrict__ s_plane, int ey, int ex, int tid, const float4& mdir,
    const float4& mraw, const MinimaxCoef& cf, float (&agg0)[W * W], float (&cen0)[W * W],
    float (&agg1)[W * W], float (&cen1)[W * W], const HOOK& hook = HOOK{}) {
    using Gm = FwdGeom<W, EXT_W, EXT_H>;
    constexpr int H = Gm::H, G = Gm::G;
    constexpr int NT = PSTRIDE > 0 ? PSTRIDE : Gm::NT;  // plane stride
    constexpr int NP = PASS == 2 ? 2 : 1;
    const bool mzero = U8 && mdir.w < 0.0f;
    const uint64_t mzero_wave = U8 ? __builtin_amdgcn_ballot_w64(mzero) : 0;
    const AtanCoef ac = atan_coef();

    auto terms = [&](int q, float (&v)[NP]) {
        if constexpr (U8) {
            const float4 b = px.dir[q];
            const float ib = DIST == kExact ? 0.0f : px.inv[q];
            float th = 0.0f, l2 = 0.0f;
            pair_u8<KIND, DIST, PASS != 1, PASS != 0>(mdir, mraw.w, mzero, mzero_wave, b, ib, cf,
                                                      ac, th, l2);
            v[0] = PASS == 1 ? l2 : th;
            if constexpr (PASS == 2) v[NP - 1] = l2;
        } else if constexpr (PASS == 1) {
            v[0] = l2_term(mraw, px.raw[q]);
        } else if constexpr (PASS == 0) {
            v[0] = pair_term<KIND, DIST, U8>(mdir, mraw, px.dir[q], px.raw[q], cf, ac);
        } else {
            const float4 rb = px.raw[q];
            v[0] = pair_term<KIND, DIST, U8>(mdir, mraw, px.dir[q], rb, cf, ac);
            v[NP - 1] = l2_term(mraw, rb);
        }
    };
    float self[NP];
    if constexpr (PASS == 1) {
        self[0] = 0.0f;
    } else {
        self[0] = self_term<KIND, DIST>(cf);
        if constexpr (NP == 2) self[NP - 1] = 0.0f;
    }

    float R[NP][G][W];  // R[k][dy + 2h][s + 2h]: sum of G_p(dy, s .. s + w - 1), term k
#pragma unroll
    for (int g = 0; g <= 2 * H; ++g) {
        float own[NP][G], up[NP][G];
#pragma unroll
        for (int dx = -2 * H; dx <= 2 * H; ++dx) {
#pragma unroll
            for (int k = 0; k < NP; ++k) own[k][dx + 2 * H] = 0.0f;
            if (g == 0 && dx <= 0) continue;
            const int py = ey + g, px_ = ex + dx;
            if (!GUARD || (py < EXT_H && px_ >= 0 && px_ < EXT_W)) {
                float v[NP];
                terms(tid + g * EXT_W + dx, v);
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    own[k][dx + 2 * H] = v[k];
                    s_plane[(k * G + dx + 2 * H) * NT + tid] = v[k];
                }
            }
        }
        hook.before(g);
        __syncthreads();
        hook.after(g);
#pragma unroll
        for (int dx = -2 * H; dx <= 2 * H; ++dx) {
#pragma unroll
            for (int k = 0; k < NP; ++k) up[k][dx + 2 * H] = 0.0f;
            if (g == 0 && dx >= 0) continue;
            const int py = ey - g, px_ = ex + dx;
            if (!GUARD || (py >= 0 && px_ >= 0 && px_ < EXT_W))
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    up[k][dx + 2 * H] = s_plane[(k * G + 2 * H - dx) * NT + tid - g * EXT_W + dx];
        }
        if constexpr (CEN) {
            if (g <= H) {
                // offset (g, dx) from p is the centre of window (-g, -dx),
                // offset (-g, dx) the centre of window (g, -dx)
#pragma unroll
                for (int dx = -H; dx <= H; ++dx) {
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        float(&cen)[W * W] = k == 0 ? cen0 : cen1;
                        const float vo = g > 0 || dx > 0
                                             ? own[k][dx + 2 * H]
                                             : (dx < 0 ? up[k][dx + 2 * H] : self[k]);
                        cen[(H - g) * W + (H - dx)] = vo;
                        if (g > 0) cen[(H + g) * W + (H - dx)] = up[k][dx + 2 * H];
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if (g == 0) {
                float row[G];
#pragma unroll
                for (int j = 0; j < G; ++j)
                    row[j] = j < 2 * H ? up[k][j] : (j == 2 * H ? self[k] : own[k][j]);
                row_sums<W>(row, R[k][2 * H]);
            } else {
                row_sums<W>(own[k], R[k][2 * H + g]);
                row_sums<W>(up[k], R[k][2 * H - g]);
            }
            if constexpr (!std::is_same_v<HOOK, NoPlaneHook>) {
                // a hook brings loops (control flow) between the row groups,
                // past which the compiler would sink these sums to their use
                // after the sweep, keeping every raw pair term live until
                // then: the sums are made here
                pin_values(R[k][2 * H + g]);
                if (g > 0) pin_values(R[k][2 * H - g]);
            }
        }
        __syncthreads();
    }
    {
        // window aggregates: column sums of the row sums, top to bottom
#pragma clang fp contract(off)
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            float(&agg)[W * W] = k == 0 ? agg0 : agg1;
#pragma unroll
            for (int uy = -H; uy <= H; ++uy) {
#pragma unroll
                for (int ux = -H; ux <= H; ++ux) {
                    const int s = -H - ux + 2 * H;
                    float acc = R[k][-H - uy + 2 * H][s];
#pragma unroll
                    for (int dy = -H - uy + 1; dy <= H - uy; ++dy) acc += R[k][dy + 2 * H][s];
                    agg[(uy + H) * W + (ux + H)] = acc;
                }
            }
        }
    }
}

// One term (angular if !L2PASS, else L2), optionally with the centre terms.
template <int W, int KIND, int DIST, bool U8, int EXT_W, int EXT_H, bool L2PASS, bool CEN,
          bool GUARD = true>
__device__ __forceinline__ void member_aggregates_c(const TilePix& px, float* __restrict__ s_plane,
                                                    int ey, int ex, int tid, const float4& mdir,
                                                    const float4& mraw, const MinimaxCoef& cf,
                                                    float (&agg)[W * W], float (&cen)[W * W]) {
    float u0[W * W], u1[W * W];
    member_aggregates_x<W, KIND, DIST, U8, EXT_W, EXT_H, L2PASS ? 1 : 0, CEN, GUARD>(
        px, s_plane, ey, ex, tid, mdir, mraw, cf, agg, cen, u0, u1);
}

template <int W, int KIND, int DIST, bool U8, int EXT_W, int EXT_H, bool L2PASS,
          bool GUARD = true>
__device__ __forceinline__ void member_aggregates(const TilePix& px, float* __restrict__ s_plane,
                                                  int ey, int ex, int tid, const float4& mdir,
                                                  const float4& mraw, const MinimaxCoef& cf,
                                                  float (&agg)[W * W]) {
    float unused[W * W];
    member_aggregates_c<W, KIND, DIST, U8, EXT_W, EXT_H, L2PASS, false, GUARD>(
        px, s_plane, ey, ex, tid, mdir, mraw, cf, agg, unused);
}

// Objective of one member: BVDF (eq. 2) A; DDF A^(1-p) D^p (p = 1/2 orders as
// the product of eq. 3).  objective_value is the objective itself;
// ObjectiveKey gives, per launch, a monotone image of it used for comparisons:
// A (BVDF, p = 0), D (p = 1), A*D (p = 1/2), A^3 D (p = 1/4) or
// (1-p) log2 A + p log2 D.  The mode depends only on p, so it is uniform.
template <int KIND>
__device__ __forceinline__ float objective_value(float A, float D, float p) {
    if (KIND == kBVDF || p == 0.0f) return A;
    if (p == 1.0f) return D;
    return exp2f(fmaf(1.0f - p, log2f(A), p * log2f(D)));
}

enum ObjMode { kObjA = 0, kObjD = 1, kObjProd = 2, kObjQuarter = 3, kObjLog = 4 };

template <int KIND>
__device__ __forceinline__ int objective_mode(float p) {
    if (KIND == kACW) return kObjProd;  // eq. (3)
    if (KIND == kBVDF || p == 0.0f) return kObjA;
    if (p == 1.0f) return kObjD;
    if (p == 0.5f) return kObjProd;
    if (p == 0.25f) return kObjQuarter;
    return kObjLog;
}

// Order bits of the objective of all n members, one uniform branch on the
// mode (outside the member loop, so no member pays for the other modes).
// Every mode but the logarithmic one yields a non-negative value (sums and
// products of non-negative terms, never -0 or NaN), whose binary32 bit
// pattern already orders like the value; the logarithmic mode can be
// negative and takes the sign-aware order_key.
template <int NW>
__device__ __forceinline__ void objective_key_bits(int mode, float p, const float (&A)[NW],
                                                   const float (&D)[NW], uint32_t (&kb)[NW]) {
    if (mode == kObjA) {
#pragma unroll
        for (int u = 0; u < NW; ++u) kb[u] = __float_as_uint(A[u]);
    } else if (mode == kObjD) {
#pragma unroll
        for (int u = 0; u < NW; ++u) kb[u] = __float_as_uint(D[u]);
    } else if (mode == kObjProd) {
#pragma unroll
        for (int u = 0; u < NW; ++u) kb[u] = __float_as_uint(A[u] * D[u]);
    } else if (mode == kObjQuarter) {
#pragma unroll
        for (int u = 0; u < NW; ++u) kb[u] = __float_as_uint((A[u] * A[u]) * (A[u] * D[u]));
    } else {
        const float q = 1.0f - p;
#pragma unroll
        for (int u = 0; u < NW; ++u)
            kb[u] = order_key(fmaf(q, __builtin_amdgcn_logf(A[u]), p * __builtin_amdgcn_logf(D[u])));
    }
}

}  // namespace odf
