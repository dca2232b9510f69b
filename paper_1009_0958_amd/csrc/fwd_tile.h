// fwd_tile.h -- one output tile of the forward filter (BVDF / DDF), shared
// by the per-image kernels and the persistent batch kernels.
//
// Per workgroup tile (aggregates.h describes a2/a3):
//   a1  load + prepare the pixel (direction, norms / chromaticity sums) -> LDS
//   a2  pair terms, each unordered pixel pair once, via LDS row-group planes
//   a3  canonical-order box sums -> aggregates of every (member, window)
//   a4  objective (BVDF: A; DDF: A^(1-p) D^p compared as (1-p) log2 A + p log2 D)
//       and argmin by a 64-bit LDS atomicMin of (ordered objective, member
//       index): the smallest objective wins, ties go to the lowest index,
//       independent of the order of the atomics; then the selected member is
//       copied to the output.
#pragma once

#include <type_traits>

#include "aggregates.h"
#include "canon.h"
#include "odf_internal.h"

namespace odf {

// LDS of one forward tile.  STAGE: the 5x5 DDF path parks the angle part of
// every (window, member) objective in LDS during the L2 pass instead of
// keeping 25 aggregates live in registers, which lets it use 1024-thread tiles;
// CWDDF^k parks its weighted angle sum the same way (50 aggregates).
// NKEY: argmin keys per window (4 for ACWDDF: eq. 3 and three levels of eq. 9).
// NPL: plane sets (2 when the angular and L2 terms are swept together).
// U8: uint8 layout (pair_terms.h): no raw array, aux2 in inv for MINIMAX and
// RGB.  HALO: the key array covers every window centre a member of the
// extended tile belongs to (rows -2h .. EXT_H - 1 of the output tile, stride
// EXT_W), so each member reaches its windows' keys at fixed offsets and no
// window needs a bounds test; the others keep one key per output pixel.
// The unguarded sweep (aggregates.h) reads up to 2h rows + 2h past dir (and
// raw, inv) and as far before plane: the member order below keeps both inside
// the struct, which fwd_tile checks.  stage holds one value per (window, output
// pixel): stage[u][cy][cx].  CANON: the direction in dir is the canonical one
// of canon.h, and rgb keeps each pixel's raw colour (bytes 0..2) for the copy.
template <int W, int EXT_W, int EXT_H, bool AGG, bool STAGE, int NKEY, int NPL, bool U8,
          bool INV, bool CANON>
struct FwdShared {
    using Gm = FwdGeom<W, EXT_W, EXT_H>;
    static constexpr bool HALO = !AGG && (U8 || W >= 5);
    static constexpr int KEYN =
        HALO ? (Gm::TH + 4 * Gm::H) * EXT_W + 2 * Gm::H : Gm::TH * Gm::TW;
    float4 dir[Gm::NT];
    float4 raw[U8 ? 1 : Gm::NT];
    float inv[INV ? Gm::NT : 1];
    uint32_t rgb[CANON ? Gm::NT : 1];  // CANON: the raw uint8 colour, for the output copy
    float plane[NPL * Gm::G * Gm::NT];
    unsigned long long key[AGG ? 1 : NKEY * KEYN];
    float stage[STAGE ? Gm::NW * Gm::TH * Gm::TW : 1];

    // key slot of the window centred on output pixel (cy, cx), tile-local
    static __device__ __forceinline__ int key_index(int cy, int cx) {
        return HALO ? (cy + 2 * Gm::H) * EXT_W + cx + 2 * Gm::H : cy * Gm::TW + cx;
    }
};

// The objective key of the windows whose angle part is staged (5x5 and larger
// DDF), in two steps: the part of A alone -- A (p = 0 or 1/2), A^3 (p = 1/4) or
// (1 - p) log2 A -- then its combination with D.  Every form of these filters
// (tile, strip, batch) forms the key this way, so they select bit for bit alike.
template <int MODE>
__device__ __forceinline__ float staged_part(float a, float p) {
    if constexpr (MODE == kObjQuarter) return (a * a) * a;  // A^3 D
    else if constexpr (MODE == kObjLog) return (1.0f - p) * __builtin_amdgcn_logf(a);
    else return a;  // A, A*D
}
template <int MODE>
__device__ __forceinline__ uint32_t staged_key_bits(float part, float d, float p) {
    if constexpr (MODE == kObjA) return __float_as_uint(part);
    else if constexpr (MODE == kObjD) return __float_as_uint(d);
    else if constexpr (MODE == kObjLog) return order_key(fmaf(p, __builtin_amdgcn_logf(d), part));
    else return __float_as_uint(part * d);  // non-negative: the bits order like the values
}

template <int W, int KIND, bool AGG>
constexpr bool stage_angle_part() {
    return W >= 5 && (KIND == kDDF || KIND == kCW) && !AGG;
}

// 3x3 DDF and ACWDDF sweep the angular and L2 terms together (PASS 2 of
// member_aggregates_x); 5x5 keeps two sweeps (register budget).
template <int W, int KIND>
constexpr bool fused_sweep() {
    return W == 3 && KIND != kBVDF && KIND != kCWV;
}

template <int W, int KIND, int DIST, bool U8, int EXT_W, int EXT_H, bool AGG>
using FwdSharedFor = FwdShared<W, EXT_W, EXT_H, AGG, stage_angle_part<W, KIND, AGG>(),
                               KIND == kACW ? 4 : 1, fused_sweep<W, KIND>() ? 2 : 1, U8,
                               U8 && DIST != kExact, U8 && KIND == kBVDF>;

// Filter one output tile whose top-left output pixel is (ty0, tx0) of image b.
// Every thread of the workgroup must call it (it synchronises); tid is the
// thread's index in the workgroup.
template <int W, int KIND, int DIST, bool U8, int EXT_W, int EXT_H, bool AGG>
__device__ __forceinline__ void fwd_tile(FwdSharedFor<W, KIND, DIST, U8, EXT_W, EXT_H, AGG>& sh,
                                         const FwdParams& prm, int b, int ty0, int tx0, int tid) {
    using Gm = FwdGeom<W, EXT_W, EXT_H>;
    using Sh = FwdSharedFor<W, KIND, DIST, U8, EXT_W, EXT_H, AGG>;
    constexpr int H = Gm::H, NW = Gm::NW, TW = Gm::TW, TH = Gm::TH, NT = Gm::NT;
    constexpr bool INV = U8 && DIST != kExact;
    // BVDF on uint8 pixels takes the canonical direction of canon.h (the
    // angular sweep alone decides, so collinear colours tie bit for bit); the
    // DDF family keeps the raw vector, whose dot product its L2 term reuses
    constexpr bool CANON = U8 && KIND == kBVDF;
    constexpr int KEYN = Sh::KEYN;
    // the unguarded sweep's reads past the pixel arrays and before the planes
    // stay inside this struct
    constexpr size_t kOver = 2 * H * EXT_W + 2 * H;
    static_assert(offsetof(Sh, dir) + (NT + kOver) * sizeof(float4) <= sizeof(Sh), "dir");
    static_assert(U8 || offsetof(Sh, raw) + (NT + kOver) * sizeof(float4) <= sizeof(Sh), "raw");
    static_assert(!INV || offsetof(Sh, inv) + (NT + kOver) * sizeof(float) <= sizeof(Sh), "inv");
    static_assert(offsetof(Sh, plane) >= kOver * sizeof(float), "plane");
    float4* s_dir = sh.dir;
    float* s_plane = sh.plane;
    unsigned long long* s_key = sh.key;
    const TilePix px{sh.dir, sh.raw, sh.inv};

    const int ey = tid / EXT_W, ex = tid - ey * EXT_W;
    const int M = prm.M, N = prm.N;

    // a1: own extended pixel, replicated border
    float4 mdir, mraw;
    {
        const int gy = min(max(ty0 - H + ey, 0), M - 1);
        const int gx = min(max(tx0 - H + ex, 0), N - 1);
        const int pix = (b * M + gy) * N + gx;  // B*M*N < 2^31 (checked on the host)
        float x0, x1, x2;
        if (U8) {
            const uint8_t* s = static_cast<const uint8_t*>(prm.img) + (size_t)pix * 3;
            const uint32_t c0 = s[0], c1 = s[1], c2 = s[2];
            x0 = c0; x1 = c1; x2 = c2;
            if constexpr (CANON) {
                float d0, d1, d2;
                canonical_direction(c0, c1, c2, d0, d1, d2);
                prepare_pixel<DIST, U8, true>(x0, x1, x2, mdir, mraw, d0, d1, d2);
                sh.rgb[tid] = c0 | (c1 << 8) | (c2 << 16);
            } else {
                prepare_pixel<DIST, U8>(x0, x1, x2, mdir, mraw);
            }
        } else {
            const float* s = static_cast<const float*>(prm.img) + (size_t)pix * 3;
            x0 = s[0]; x1 = s[1]; x2 = s[2];
            prepare_pixel<DIST, U8>(x0, x1, x2, mdir, mraw);
        }
        s_dir[tid] = mdir;
        if constexpr (!U8) sh.raw[tid] = mraw;
        if constexpr (INV) sh.inv[tid] = mraw.w;
    }
    constexpr int NKEY = KIND == kACW ? 4 : 1;
    if (!AGG)
        for (int i = tid; i < NKEY * KEYN; i += NT) s_key[i] = ~0ull;
    __syncthreads();

    // a2 + a3 (ACWDDF also keeps each member's terms with the window centres)
    float A[NW], D[NW];
    float cA[NW], cD[NW];
    if constexpr (KIND == kCWV) {
#pragma unroll
        for (int u = 0; u < NW; ++u) A[u] = cA[u] = 0.0f;  // no angle term
    } else if constexpr (fused_sweep<W, KIND>())
        member_aggregates_x<W, KIND, DIST, U8, EXT_W, EXT_H, 2, centre_weighted(KIND),
                            false>(px, s_plane, ey, ex, tid, mdir, mraw, prm.coef, A, cA, D, cD);
    else
        member_aggregates_c<W, KIND, DIST, U8, EXT_W, EXT_H, false, centre_weighted(KIND),
                            false>(px, s_plane, ey, ex, tid, mdir, mraw, prm.coef, A, cA);
    if constexpr (stage_angle_part<W, KIND, AGG>() && KIND == kCW) {
        // weighted angle sum A + (w_d(k) - 1) cA of each window -> LDS, then the
        // L2 pass with its centre terms
        const float w1 = prm.acw_wm1[0];
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            const int cy = ey - u / W, cx = ex - u % W;
            if (cy < 0 || cy >= TH || cx < 0 || cx >= TW) continue;
            sh.stage[u * (TH * TW) + cy * TW + cx] = fmaf(w1, cA[u], A[u]);
        }
        member_aggregates_c<W, KIND, DIST, U8, EXT_W, EXT_H, true, true, false>(
            px, s_plane, ey, ex, tid, mdir, mraw, prm.coef, D, cD);
    } else if constexpr (stage_angle_part<W, KIND, AGG>()) {
        // angle part of each objective -> LDS, then the L2 pass
        const int mode = objective_mode<KIND>(prm.p);
        const float p = prm.p;
        auto stage_parts = [&](auto mode_c) {
            constexpr int MODE = decltype(mode_c)::value;
#pragma unroll
            for (int u = 0; u < NW; ++u) {
                const int cy = ey - u / W, cx = ex - u % W;
                if (cy < 0 || cy >= TH || cx < 0 || cx >= TW) continue;
                sh.stage[u * (TH * TW) + cy * TW + cx] = staged_part<MODE>(A[u], p);
            }
        };
        if (mode == kObjQuarter) stage_parts(std::integral_constant<int, kObjQuarter>{});
        else if (mode == kObjLog) stage_parts(std::integral_constant<int, kObjLog>{});
        else stage_parts(std::integral_constant<int, kObjA>{});
        member_aggregates<W, KIND, DIST, U8, EXT_W, EXT_H, true, false>(px, s_plane, ey, ex, tid,
                                                                       mdir, mraw, prm.coef, D);
    } else if constexpr (fused_sweep<W, KIND>()) {
        ;  // D and cD came with the angular sweep
    } else if (KIND != kBVDF) {
        member_aggregates_c<W, KIND, DIST, U8, EXT_W, EXT_H, true, centre_weighted(KIND),
                            false>(px, s_plane, ey, ex, tid, mdir, mraw, prm.coef, D, cD);
    } else {
#pragma unroll
        for (int u = 0; u < NW; ++u) D[u] = 0.0f;
    }

    // Window u of this member is centred on output pixel (ey - u / W, ex - u % W)
    // of the tile.  Windows outside the output tile (or the image) hold
    // meaningless aggregates (unguarded sweep): without HALO they are
    // skipped, with HALO their keys land in slots no output pixel reads.
    // With HALO a wave skips window u only when it lies outside the output
    // tile's rows for all of the wave's rows (a scalar test).
    constexpr int RW = 64 / EXT_W;
    const int wrow0 = __builtin_amdgcn_readfirstlane(ey);
    auto window_ok = [&](int u) {
        const int cy = ey - u / W, cx = ex - u % W;
        if (Sh::HALO) return wrow0 + RW - 1 - u / W >= 0 && wrow0 - u / W < TH;
        return cy >= 0 && cy < TH && cx >= 0 && cx < TW && ty0 + cy < M && tx0 + cx < N;
    };
    // the key slot of window u: a fixed offset from the member's own slot
    auto key_slot = [&](int u) {
        return Sh::HALO ? tid + (2 * H - u / W) * EXT_W + 2 * H - u % W
                        : Sh::key_index(ey - u / W, ex - u % W);
    };

    // a4: objective of this member in every window of the tile containing it
    if (AGG) {
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            const int cy = ey - u / W;  // window centre, tile-local
            const int cx = ex - u % W;
            if (cy < 0 || cy >= TH || cx < 0 || cx >= TW) continue;
            if (ty0 + cy >= M || tx0 + cx >= N) continue;
            const size_t o = (((size_t)b * M + ty0 + cy) * N + tx0 + cx) * NW + u;
            prm.dbg_A[o] = A[u];
            if (prm.dbg_D) prm.dbg_D[o] = D[u];
            if (prm.dbg_O) prm.dbg_O[o] = objective_value<KIND>(A[u], D[u], prm.p);
        }
    } else if constexpr (stage_angle_part<W, KIND, AGG>() && KIND == kCW) {
        // the staged weighted angle sum times the weighted L2 sum (the stage
        // index stays in range as in the DDF loop below)
        const float w1 = prm.acw_wm1[0];
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            if (!window_ok(u)) continue;
            const int cy = ey - u / W, cx = ex - u % W;
            const float o = sh.stage[u * (TH * TW) + cy * TW + cx] * fmaf(w1, cD[u], D[u]);
            atomicMin(&s_key[key_slot(u)],
                      ((unsigned long long)__float_as_uint(o) << 32) | (unsigned)u);
        }
    } else if constexpr (stage_angle_part<W, KIND, AGG>()) {
        // the staged angle part with D; one copy of the key loop per
        // objective mode (a uniform branch outside the member loop)
        const int mode = objective_mode<KIND>(prm.p);
        const float p = prm.p;
        auto stage_keys = [&](auto mode_c) {
            constexpr int MODE = decltype(mode_c)::value;
#pragma unroll
            for (int u = 0; u < NW; ++u) {
                // with HALO every lane of a wave that does not skip window u
                // reads stage, also for a window outside the output tile: as
                // cy runs over [-(u / W), EXT_H - 1 - u / W] and cx over
                // [-(u % W), EXT_W - 1 - u % W], the index stays in
                // [0, NW TH TW), and the key lands in a slot no output pixel
                // reads
                if (!window_ok(u)) continue;
                const int cy = ey - u / W, cx = ex - u % W;
                const float part = sh.stage[u * (TH * TW) + cy * TW + cx];
                const uint32_t bits = staged_key_bits<MODE>(part, D[u], p);
                const unsigned long long key = ((unsigned long long)bits << 32) | (unsigned)u;
                atomicMin(&s_key[key_slot(u)], key);
            }
        };
        if (mode == kObjA) stage_keys(std::integral_constant<int, kObjA>{});
        else if (mode == kObjD) stage_keys(std::integral_constant<int, kObjD>{});
        else if (mode == kObjLog) stage_keys(std::integral_constant<int, kObjLog>{});
        else stage_keys(std::integral_constant<int, kObjProd>{});
    } else if constexpr (KIND == kACW) {
        // eq. (3) and the centre-weighted objectives of eq. (9): the weight
        // w_d(k) of the centre adds (w_d(k) - 1) times the centre term
        const float w1 = prm.acw_wm1[0], w2 = prm.acw_wm1[1], w3 = prm.acw_wm1[2];
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            if (!window_ok(u)) continue;
            const int ci = key_slot(u);
            const float o0 = A[u] * D[u];
            const float o1 = fmaf(w1, cA[u], A[u]) * fmaf(w1, cD[u], D[u]);
            const float o2 = fmaf(w2, cA[u], A[u]) * fmaf(w2, cD[u], D[u]);
            const float o3 = fmaf(w3, cA[u], A[u]) * fmaf(w3, cD[u], D[u]);
            // products of non-negative sums: the bit patterns order like the values
            const unsigned long long uu = (unsigned)u;
            atomicMin(&s_key[ci], ((unsigned long long)__float_as_uint(o0) << 32) | uu);
            atomicMin(&s_key[KEYN + ci], ((unsigned long long)__float_as_uint(o1) << 32) | uu);
            atomicMin(&s_key[2 * KEYN + ci], ((unsigned long long)__float_as_uint(o2) << 32) | uu);
            atomicMin(&s_key[3 * KEYN + ci], ((unsigned long long)__float_as_uint(o3) << 32) | uu);
        }
    } else if constexpr (KIND == kCW || KIND == kCWV) {
        // one centre-weighted filter at one level (weight w_d(k) - 1 = acw_wm1[0]):
        // CWDDF^k the weighted product, CWVMF^k (eq. 9) the weighted L2 sum
        const float w1 = prm.acw_wm1[0];
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            if (!window_ok(u)) continue;
            const float dw = fmaf(w1, cD[u], D[u]);
            const float o = KIND == kCWV ? dw : fmaf(w1, cA[u], A[u]) * dw;
            atomicMin(&s_key[key_slot(u)],
                      ((unsigned long long)__float_as_uint(o) << 32) | (unsigned)u);
        }
    } else {
        uint32_t kb[NW];
        objective_key_bits<NW>(objective_mode<KIND>(prm.p), prm.p, A, D, kb);
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            if (!window_ok(u)) continue;
            atomicMin(&s_key[key_slot(u)], ((unsigned long long)kb[u] << 32) | (unsigned)u);
        }
    }
    if (AGG) return;
    __syncthreads();

    // write the selected member of every window of the tile: the thread at the
    // window's centre writes it (the extended tile covers the output tile)
    {
        const int cy = ey - H, cx = ex - H;
        const int gy = ty0 + cy, gx = tx0 + cx;
        if (cy < 0 || cy >= TH || cx < 0 || cx >= TW || gy >= M || gx >= N) return;
        const int ki = Sh::key_index(cy, cx);
        int u = min((int)(s_key[ki] & 0xffu), NW - 1);
        if constexpr (KIND == kACW) {
            // switch: S = sum over the three levels of A(y_k, x_d) L2(y_k, x_d);
            // the eq. (3) selection if S > T, else the centre
            const int c = (cy + H) * EXT_W + cx + H;
            const float4 cd = s_dir[c];
            const AtanCoef ac = atan_coef();
            float S = 0.0f;
#pragma unroll
            for (int j = 1; j <= 3; ++j) {
                const int uj = min((int)(s_key[j * KEYN + ki] & 0xffu), NW - 1);
                const int m = (cy + uj / W) * EXT_W + cx + uj % W;
                if constexpr (U8) {
                    const float4 md = s_dir[m];
                    float th, l2;
                    const bool mz = md.w < 0.0f;
                    pair_u8<KIND, DIST, true, true>(md, INV ? sh.inv[m] : 0.0f, mz,
                                                    __builtin_amdgcn_ballot_w64(mz), cd,
                                                    INV ? sh.inv[c] : 0.0f, prm.coef, ac, th,
                                                    l2);
                    S += th * l2;
                } else {
                    const float4 cr = sh.raw[c];
                    S += pair_term<KIND, DIST, U8>(s_dir[m], sh.raw[m], cd, cr, prm.coef,
                                                   ac) *
                         l2_term(sh.raw[m], cr);
                }
            }
            if (!(S > prm.acw_T)) u = (NW - 1) / 2;
        }
        const int sel = (cy + u / W) * EXT_W + cx + u % W;
        const int pix = (b * M + gy) * N + gx;
        if constexpr (CANON) {
            // the canonical direction is not the value: the raw colour kept in rgb
            const uint32_t v = sh.rgb[sel];
            uint8_t* o = static_cast<uint8_t*>(prm.out) + (size_t)pix * 3;
            o[0] = (uint8_t)v; o[1] = (uint8_t)(v >> 8); o[2] = (uint8_t)(v >> 16);
        } else if (U8) {
            // the raw value is the direction, or 0 for the zero pixel
            const float4 d = s_dir[sel];
            const bool z = d.w < 0.0f;
            uint8_t* o = static_cast<uint8_t*>(prm.out) + (size_t)pix * 3;
            o[0] = z ? 0 : (uint8_t)d.x; o[1] = z ? 0 : (uint8_t)d.y; o[2] = z ? 0 : (uint8_t)d.z;
        } else {
            const float4 r = sh.raw[sel];
            float* o = static_cast<float*>(prm.out) + (size_t)pix * 3;
            o[0] = r.x; o[1] = r.y; o[2] = r.z;
        }
        if (prm.idx) prm.idx[pix] = (uint8_t)u;
    }
}

}  // namespace odf
