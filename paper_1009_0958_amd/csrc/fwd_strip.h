// fwd_strip.h -- the strip form of the forward filter (BVDF, DDF and the
// centre-weighted kinds): one workgroup filters a column strip of output
// pixels, walking down it band by band, instead of one output tile with a halo
// on all four sides.
//
// A band is EXT_W x BH member pixels (one thread each).  Each member's offset
// grid is swept exactly as in the tile form (aggregates.h: own terms of row
// group g published in LDS planes, the mirrored terms of row -g read back),
// but the planes of the band's last g rows are kept in LDS for the next band,
// whose first g rows read them instead of re-evaluating those pair terms, and
// the argmin keys of the windows that the next band's members still belong
// to stay in LDS as well.  So every unordered pixel pair of the strip is
// evaluated once per strip: the halo is recomputed across the strip's two
// vertical edges (EXT_W / TW) and over its first 2h rows, not at every tile
// boundary (the 32 x 16 tile of the 5x5 filters evaluates 1.52 times its
// output pixels' pair terms, a 32-wide strip of 8 bands 1.18 times).
//
// Every member's aggregates come out of the same summation tree as in the
// tile form, so the strip form is bitwise equal to it.
#pragma once

#include "fwd_tile.h"

namespace odf {

template <int W, int EXT_W, int BH>
struct StripGeom {
    static constexpr int H = W / 2;
    static constexpr int NW = W * W;
    static constexpr int G = 4 * H + 1;
    static constexpr int TW = EXT_W - 2 * H;    // output columns
    static constexpr int NT = EXT_W * BH;       // threads: one per member of a band
    static constexpr int RING = BH + 2 * H;     // pixel rows a band reads
    static constexpr int PL = RING * EXT_W;     // plane stride: 2h carried rows + the band
    // output rows of a strip of nb bands
    static constexpr int rows(int nb) { return nb * BH - 2 * H; }
    static constexpr int CROWS = H * (4 * H + 2) / 2;  // carried rows, summed over g = 1 .. 2h
    // key slots: window centres on band rows -h .. BH - 1 + h (ring row = centre
    // row + h), stride EXT_W, + 2h slots that windows past the last column reach
    static constexpr int KEYN = RING * EXT_W + 2 * H;
    static constexpr int KCARRY = 2 * H * EXT_W + 2 * H;  // slots handed to the next band
};

// LDS of one strip workgroup.  NPL: planes swept together (2 for the fused
// angle + L2 sweep of the 3x3 DDF family); NTERM: carried plane sets (one per
// term); NKEY: argmin keys per window (4 for ACWDDF: eq. 3 and three levels of
// eq. 9), each set a ring of KEYN slots.
template <int W, int KIND, int DIST, bool U8, int EXT_W, int BH>
struct StripShared {
    using Gm = StripGeom<W, EXT_W, BH>;
    static constexpr bool INV = U8 && DIST != kExact;
    static constexpr int NPL = fused_sweep<W, KIND>() ? 2 : 1;
    static constexpr int NTERM = (KIND == kBVDF || KIND == kCWV) ? 1 : 2;
    static constexpr int NKEY = KIND == kACW ? 4 : 1;
    static constexpr int NPIX = Gm::PL + 2 * Gm::H;  // + the reads past the last row
    float4 dir[NPIX];
    float4 raw[U8 ? 1 : NPIX];
    float inv[INV ? NPIX : 1];
    // plane rows and carried rows are copied as float4: both 16-byte aligned
    alignas(16) float plane[NPL * Gm::G * Gm::PL + 4];
    alignas(16) float carry[NTERM * Gm::G * Gm::CROWS * EXT_W];
    unsigned long long key[NKEY * Gm::KEYN];
};

// Plane hook of one sweep (aggregates.h): in row group g >= 1 it copies the
// planes of the previous band's last g rows, kept in carry, to the g rows
// above the band (before the barrier that publishes the band's own terms),
// and after that barrier keeps this band's last g rows for the next band.
// plane points at ring row 0 (the band starts at ring row 2h); NP planes of
// stride PL.  One float4 per thread and step: carry holds, per g, NP * g rows
// of EXT_W floats (plane by plane, row by row).
template <int EXT_W, int BH, int H, int NP, int PL, int NT>
struct StripCarry {
    float* plane;
    float* carry;
    int tid;
    static_assert(EXT_W % 4 == 0 && PL % 4 == 0, "float4 rows");
    static constexpr int Q = EXT_W / 4;  // float4 per row
    static constexpr int off(int g) { return NP * EXT_W * (g - 1) * g / 2; }
    template <bool IN>
    __device__ __forceinline__ void copy(int g, int row0) const {
        const int n = NP * g * Q;
        for (int i = tid; i < n; i += NT) {
            const int q = i / Q, c = i - q * Q;  // row q of the g NP carried rows
            const int d = q / g, r = q - d * g;
            float4* pl = reinterpret_cast<float4*>(plane + d * PL + (row0 + r) * EXT_W) + c;
            float4* cr = reinterpret_cast<float4*>(carry + off(g)) + i;
            if (IN) *pl = *cr;
            else *cr = *pl;
        }
    }
    __device__ __forceinline__ void before(int g) const {
        if (g > 0) copy<true>(g, 2 * H - g);
    }
    __device__ __forceinline__ void after(int g) const {
        if (g > 0) copy<false>(g, 2 * H + BH - g);
    }
};

// The classes with a strip form: BVDF and DDF at 3x3, 5x5 and 7x7, BVDF at
// 9x9 on uint8 (the float32 9x9 strip and the 9x9 DDF strip, with its second
// set of carried planes, would not fit the 160 KiB of LDS of a CU), and the
// centre-weighted kinds (ACWDDF, CWDDF^k, CWVMF^k) at 3x3 to 7x7 (7x7 ACWDDF: 152 KB of
// LDS for float32, within a CU).
template <int W, int KIND, bool U8>
constexpr bool strip_form() {
    if (centre_weighted(KIND)) return W == 3 || W == 5 || W == 7;
    if (KIND != kBVDF && KIND != kDDF) return false;
    return W == 3 || W == 5 || W == 7 || (W == 9 && KIND == kBVDF && U8);
}

// Occupancy target of a strip kernel: the waves per SIMD that its LDS allows
// (160 KiB per CU shared by whole workgroups of NT / 256 waves per SIMD), at
// most 8; the register budget is fitted to it.
constexpr int lds_waves_per_eu(size_t lds_bytes, int threads) {
    const int waves = (int)((160 * 1024) / lds_bytes) * (threads / 256);
    return waves < 1 ? 1 : (waves > 8 ? 8 : waves);
}
template <int W, int KIND, int DIST, bool U8, int EXT_W, int BH>
constexpr int strip_waves_per_eu() {
    const int lds = lds_waves_per_eu(sizeof(StripShared<W, KIND, DIST, U8, EXT_W, BH>), EXT_W * BH);
    // 5x5 ACWDDF keeps four sets of 25 aggregates (A, D and both centre terms):
    // ~146 VGPRs, one workgroup per CU; held to 128 (14 spilled) two share a CU
    // and the uint8 kernel runs 1.6x faster on 7680 x 4320
    return (W == 5 && KIND == kACW && lds > 4) ? 4 : lds;
}

// Filter the strip of image b whose first output row is s0 and first output
// column tx0 (nb bands: nb BH - 2h output rows x TW output columns, clipped to
// the image).  Bands start h rows above the strip and the first band's 2h top
// window rows lie above it (discarded); a band reads its RING pixel rows
// (replicated border), sweeps, and then writes the BH window rows its members
// completed.  Every thread of the workgroup must call it (it synchronises).
template <int W, int KIND, int DIST, bool U8, int EXT_W, int BH>
__device__ __forceinline__ void fwd_strip(StripShared<W, KIND, DIST, U8, EXT_W, BH>& sh,
                                          const FwdParams& prm, int b, int s0, int tx0, int nb) {
    using Gm = StripGeom<W, EXT_W, BH>;
    using Sh = StripShared<W, KIND, DIST, U8, EXT_W, BH>;
    constexpr int H = Gm::H, NW = Gm::NW, G = Gm::G, NT = Gm::NT, PL = Gm::PL;
    constexpr bool INV = Sh::INV;
    constexpr bool CANON = U8 && KIND == kBVDF;  // as in the tile form
    constexpr bool CEN = centre_weighted(KIND);   // the centre terms of eq. (9)
    constexpr int NKEY = Sh::NKEY, KEYN = Gm::KEYN, KCARRY = Gm::KCARRY;
    constexpr int KC = (NKEY * KCARRY + NT - 1) / NT;  // carried keys per thread
    static_assert(offsetof(Sh, plane) >= 2 * H * sizeof(float), "reads before plane");
    const int M = prm.M, N = prm.N;
    const int s_end = min(s0 + Gm::rows(nb), M);
    const TilePix px{sh.dir, sh.raw, sh.inv};
    float* const pl0 = sh.plane + 2 * H * EXT_W;  // ring row 2h: the band's first row

    // the prepared pixel (direction, and the aux2 or raw vector) at image (gy, gx)
    auto prepare_at = [&](int gy, int gx, float4& d, float4& w) {
        const int pix = (b * M + gy) * N + gx;
        if constexpr (U8) {
            const uint8_t* s = static_cast<const uint8_t*>(prm.img) + (size_t)pix * 3;
            const uint32_t c0 = s[0], c1 = s[1], c2 = s[2];
            if constexpr (CANON) {
                float d0, d1, d2;
                canonical_direction(c0, c1, c2, d0, d1, d2);
                prepare_pixel<DIST, U8, true>((float)c0, (float)c1, (float)c2, d, w, d0, d1, d2);
            } else {
                prepare_pixel<DIST, U8>((float)c0, (float)c1, (float)c2, d, w);
            }
        } else {
            const float* s = static_cast<const float*>(prm.img) + (size_t)pix * 3;
            prepare_pixel<DIST, U8>(s[0], s[1], s[2], d, w);
        }
    };

    for (int j = 0; j < nb; ++j) {
        // the thread index is laundered once per band, so that the compiler
        // derives the band's many LDS addresses inside the loop instead of
        // hoisting them all out of it (each would hold a register across it)
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const int ey = tid / EXT_W, ex = tid - ey * EXT_W;
        const int base = s0 - H + j * BH;  // image row of the band's first member row
        const int fin0 = base - H;         // image row of the first window row it completes
        if (fin0 >= s_end) break;          // uniform

        // keys of the windows the previous band's members share with this band
        // (flat index q KCARRY + k for slot k of key set q)
        unsigned long long kc[KC];
#pragma unroll
        for (int q = 0; q < KC; ++q) {
            const int i = tid + q * NT, set = NKEY == 1 ? 0 : i / KCARRY;
            kc[q] = ~0ull;
            if (j > 0 && i < NKEY * KCARRY)
                kc[q] = sh.key[set * KEYN + BH * EXT_W + i - set * KCARRY];
        }
        // a1: the band's RING pixel rows (members and the 2h rows below them)
        for (int i = tid; i < Gm::PL; i += NT) {
            const int r = i / EXT_W, c = i - r * EXT_W;
            float4 d, w;
            prepare_at(min(max(base + r, 0), M - 1), min(max(tx0 - H + c, 0), N - 1), d, w);
            sh.dir[i] = d;
            if constexpr (!U8) sh.raw[i] = w;
            if constexpr (INV) sh.inv[i] = w.w;
        }
        __syncthreads();
        for (int i = tid; i < NKEY * KEYN; i += NT) {
            const int set = NKEY == 1 ? 0 : i / KEYN;
            if (i - set * KEYN >= KCARRY) sh.key[i] = ~0ull;
        }
#pragma unroll
        for (int q = 0; q < KC; ++q) {
            const int i = tid + q * NT, set = NKEY == 1 ? 0 : i / KCARRY;
            if (i < NKEY * KCARRY) sh.key[set * KEYN + i - set * KCARRY] = kc[q];
        }

        const float4 mdir = sh.dir[tid];
        float4 mraw;
        if constexpr (U8) mraw = make_float4(0.0f, 0.0f, 0.0f, INV ? sh.inv[tid] : 0.0f);
        else mraw = sh.raw[tid];

        // a2 + a3: A and D (and the centre terms cA, cD of the centre-weighted kinds)
        float A[NW], D[NW], cA[NW], cD[NW];
        if constexpr (KIND == kCWV) {  // eq. (9) on the L2 term alone
#pragma unroll
            for (int u = 0; u < NW; ++u) A[u] = cA[u] = 0.0f;
            const StripCarry<EXT_W, BH, H, G, PL, NT> hd{sh.plane, sh.carry, tid};
            float u0[NW], u1[NW];
            member_aggregates_x<W, KIND, DIST, U8, EXT_W, BH, 1, true, false, PL>(
                px, pl0, ey, ex, tid, mdir, mraw, prm.coef, D, cD, u0, u1, hd);
        } else if constexpr (fused_sweep<W, KIND>()) {
            const StripCarry<EXT_W, BH, H, 2 * G, PL, NT> hk{sh.plane, sh.carry, tid};
            member_aggregates_x<W, KIND, DIST, U8, EXT_W, BH, 2, CEN, false, PL>(
                px, pl0, ey, ex, tid, mdir, mraw, prm.coef, A, cA, D, cD, hk);
        } else {
            const StripCarry<EXT_W, BH, H, G, PL, NT> hk{sh.plane, sh.carry, tid};
            member_aggregates_x<W, KIND, DIST, U8, EXT_W, BH, 0, CEN, false, PL>(
                px, pl0, ey, ex, tid, mdir, mraw, prm.coef, A, cA, D, cD, hk);
            if constexpr (KIND != kBVDF) {
                // the aggregates, not the row sums, live through the L2 sweep
                if constexpr (KIND == kCW) {
                    // CWDDF^k needs the angle sums only weighted: A + (w_d(k) - 1) cA
                    const float w1 = prm.acw_wm1[0];
#pragma unroll
                    for (int u = 0; u < NW; ++u) A[u] = fmaf(w1, cA[u], A[u]);
                    pin_values(A);
                } else {
                    pin_values(A);
                    if constexpr (CEN) pin_values(cA);
                }
                const StripCarry<EXT_W, BH, H, G, PL, NT> hd{
                    sh.plane, sh.carry + G * Gm::CROWS * EXT_W, tid};
                float u0[NW], u1[NW];
                member_aggregates_x<W, KIND, DIST, U8, EXT_W, BH, 1, CEN, false, PL>(
                    px, pl0, ey, ex, tid, mdir, mraw, prm.coef, D, cD, u0, u1, hd);
            } else {
#pragma unroll
                for (int u = 0; u < NW; ++u) D[u] = 0.0f;
            }
        }

        // a4: every window of the member; window u is centred on band row
        // ey + h - u / W, column ex + h - u % W, key slot (row + h) EXT_W + col + h
        // of each key set.  Windows past the strip's columns hold meaningless
        // aggregates and land in slots no output reads.  The member numbers are
        // formed here: as constants the compiler keeps all n of them in vector
        // registers across the band loop.
        {
            unsigned z = 0;
            asm volatile("" : "+v"(z));
            auto slot = [&](int u) { return tid + (2 * H - u / W) * EXT_W + 2 * H - u % W; };
            if constexpr (KIND == kACW) {
                // eq. (3) and the centre-weighted objectives of eq. (9), as the tile form
                const float w1 = prm.acw_wm1[0], w2 = prm.acw_wm1[1], w3 = prm.acw_wm1[2];
#pragma unroll
                for (int u = 0; u < NW; ++u) {
                    const unsigned long long uu = z + (unsigned)u;
                    const float o0 = A[u] * D[u];
                    const float o1 = fmaf(w1, cA[u], A[u]) * fmaf(w1, cD[u], D[u]);
                    const float o2 = fmaf(w2, cA[u], A[u]) * fmaf(w2, cD[u], D[u]);
                    const float o3 = fmaf(w3, cA[u], A[u]) * fmaf(w3, cD[u], D[u]);
                    const int k = slot(u);
                    atomicMin(&sh.key[k], ((unsigned long long)__float_as_uint(o0) << 32) | uu);
                    atomicMin(&sh.key[KEYN + k],
                              ((unsigned long long)__float_as_uint(o1) << 32) | uu);
                    atomicMin(&sh.key[2 * KEYN + k],
                              ((unsigned long long)__float_as_uint(o2) << 32) | uu);
                    atomicMin(&sh.key[3 * KEYN + k],
                              ((unsigned long long)__float_as_uint(o3) << 32) | uu);
                }
            } else if constexpr (KIND == kCW || KIND == kCWV) {
                // one centre-weighted filter at one level: CWDDF^k the weighted
                // product, CWVMF^k (eq. 9) the weighted L2 sum (at 5x5, A holds
                // the weighted angle sums of CWDDF^k already)
                const float w1 = prm.acw_wm1[0];
#pragma unroll
                for (int u = 0; u < NW; ++u) {
                    const float dw = fmaf(w1, cD[u], D[u]);
                    float o = dw;
                    if constexpr (KIND == kCW)
                        o = (fused_sweep<W, KIND>() ? fmaf(w1, cA[u], A[u]) : A[u]) * dw;
                    atomicMin(&sh.key[slot(u)],
                              ((unsigned long long)__float_as_uint(o) << 32) | (z + (unsigned)u));
                }
            } else {
                uint32_t kb[NW];
                const int mode = objective_mode<KIND>(prm.p);
                if constexpr (stage_angle_part<W, KIND, false>()) {
                    // the key as the tile form's staged path forms it
                    auto staged = [&](auto mode_c) {
                        constexpr int MODE = decltype(mode_c)::value;
#pragma unroll
                        for (int u = 0; u < NW; ++u)
                            kb[u] = staged_key_bits<MODE>(staged_part<MODE>(A[u], prm.p), D[u],
                                                          prm.p);
                    };
                    if (mode == kObjA) staged(std::integral_constant<int, kObjA>{});
                    else if (mode == kObjD) staged(std::integral_constant<int, kObjD>{});
                    else if (mode == kObjLog) staged(std::integral_constant<int, kObjLog>{});
                    else if (mode == kObjQuarter) staged(std::integral_constant<int, kObjQuarter>{});
                    else staged(std::integral_constant<int, kObjProd>{});
                } else {
                    objective_key_bits<NW>(mode, prm.p, A, D, kb);
                }
#pragma unroll
                for (int u = 0; u < NW; ++u)
                    atomicMin(&sh.key[slot(u)],
                              ((unsigned long long)kb[u] << 32) | (z + (unsigned)u));
            }
        }
        __syncthreads();

        // the BH window rows this band completed: ring rows 0 .. BH - 1
        {
            const int gy = fin0 + ey, gx = tx0 - H + ex;
            if (ex >= H && ex < EXT_W - H && gy >= s0 && gy < s_end && gx < N) {
                const int ki = ey * EXT_W + ex + H;
                int u = min((int)(sh.key[ki] & 0xffu), NW - 1);
                if constexpr (KIND == kACW) {
                    // switch: S = sum over the three levels of A(y_k, x_c) L2(y_k, x_c),
                    // the pixels prepared again from the image (a member may lie in the
                    // previous band's rows); the eq. (3) selection if S > T, else the
                    // centre
                    float4 cd, cw;
                    prepare_at(gy, gx, cd, cw);
                    const AtanCoef ac = atan_coef();
                    float S = 0.0f;
#pragma unroll
                    for (int q = 1; q <= 3; ++q) {
                        const int uj = min((int)(sh.key[q * KEYN + ki] & 0xffu), NW - 1);
                        float4 md, mw;
                        prepare_at(min(max(gy - H + uj / W, 0), M - 1),
                                   min(max(gx - H + uj % W, 0), N - 1), md, mw);
                        if constexpr (U8) {
                            float th, l2;
                            const bool mz = md.w < 0.0f;
                            pair_u8<KIND, DIST, true, true>(md, INV ? mw.w : 0.0f, mz,
                                                            __builtin_amdgcn_ballot_w64(mz), cd,
                                                            INV ? cw.w : 0.0f, prm.coef, ac, th,
                                                            l2);
                            S += th * l2;
                        } else {
                            S += pair_term<KIND, DIST, U8>(md, mw, cd, cw, prm.coef, ac) *
                                 l2_term(mw, cw);
                        }
                    }
                    if (!(S > prm.acw_T)) u = (NW - 1) / 2;
                }
                const int sy = min(max(gy - H + u / W, 0), M - 1);
                const int sx = min(max(gx - H + u % W, 0), N - 1);
                const int src = (b * M + sy) * N + sx;
                const int pix = (b * M + gy) * N + gx;
                if constexpr (U8) {
                    const uint8_t* s = static_cast<const uint8_t*>(prm.img) + (size_t)src * 3;
                    uint8_t* o = static_cast<uint8_t*>(prm.out) + (size_t)pix * 3;
                    o[0] = s[0]; o[1] = s[1]; o[2] = s[2];
                } else {
                    const float* s = static_cast<const float*>(prm.img) + (size_t)src * 3;
                    float* o = static_cast<float*>(prm.out) + (size_t)pix * 3;
                    o[0] = s[0]; o[1] = s[1]; o[2] = s[2];
                }
                if (prm.idx) prm.idx[pix] = (uint8_t)u;
            }
        }
    }
}

// One workgroup per strip of the launch's images (prm.strip_bands bands each),
// in the XCD-contiguous order of xcd_item: neighbouring strips share their
// overlapping columns and the cache lines that 3-byte pixels straddle in one
// XCD's L2 (HBM traffic of the 5x5 DDF strip on 7680 x 4320: 2.07 -> 1.03 times
// the algorithmic bytes, at the same speed).
template <int W, int KIND, int DIST, bool U8, int EXT_W, int BH>
__global__ void __launch_bounds__(EXT_W* BH)
    __attribute__((amdgpu_waves_per_eu(strip_waves_per_eu<W, KIND, DIST, U8, EXT_W, BH>())))
    fwd_strip_kernel(FwdParams prm) {
    __shared__ StripShared<W, KIND, DIST, U8, EXT_W, BH> sh;
    using Gm = StripGeom<W, EXT_W, BH>;
    const int t0 = flat_block(prm.grid.n);
    if (t0 < 0) return;
    const TileCoord tc = tile_coord(xcd_item(t0, prm.grid.n), prm.grid);
    const int nb = prm.strip_bands;
    fwd_strip<W, KIND, DIST, U8, EXT_W, BH>(sh, prm, tc.b, tc.ty * Gm::rows(nb), tc.tx * Gm::TW,
                                            nb);
}

template <int W, int KIND, int DIST, bool U8, int EXT_W, int BH>
static hipError_t launch_strip(const FwdParams& prm, int nb, hipStream_t stream) {
    using Gm = StripGeom<W, EXT_W, BH>;
    FwdParams q = prm;
    q.strip_bands = nb;
    const int S = Gm::rows(nb);
    q.grid = tile_grid(prm.B, (prm.N + Gm::TW - 1) / Gm::TW, (prm.M + S - 1) / S);
    hipLaunchKernelGGL((fwd_strip_kernel<W, KIND, DIST, U8, EXT_W, BH>), flat_grid(q.grid.n),
                       dim3(Gm::NT), 0, stream, q);
    return hipGetLastError();
}

// The per-image strip launch of window W (32-wide strips of nb bands of 16
// rows) for a class given at run time; each window size is instantiated in a
// translation unit of its own (fwd3s.hip .. fwd9s.hip), beside the tile ones.
template <int W, int KIND, bool U8>
static hipError_t launch_strip_class(int dist, const FwdParams& prm, int nb, hipStream_t s) {
    if constexpr (!strip_form<W, KIND, U8>()) {
        (void)dist; (void)prm; (void)nb; (void)s;
        return hipErrorInvalidValue;
    } else {
        switch (dist) {
        case kExact: return launch_strip<W, KIND, kExact, U8, 32, 16>(prm, nb, s);
        case kMinimax: return launch_strip<W, KIND, kMinimax, U8, 32, 16>(prm, nb, s);
        default: return launch_strip<W, KIND, kRgb, U8, 32, 16>(prm, nb, s);
        }
    }
}
template <int W>
static hipError_t launch_strip_w(int kind, int dist, bool u8, const FwdParams& prm, int nb,
                                 hipStream_t s) {
    if (kind == kBVDF)
        return u8 ? launch_strip_class<W, kBVDF, true>(dist, prm, nb, s)
                  : launch_strip_class<W, kBVDF, false>(dist, prm, nb, s);
    if (kind == kDDF)
        return u8 ? launch_strip_class<W, kDDF, true>(dist, prm, nb, s)
                  : launch_strip_class<W, kDDF, false>(dist, prm, nb, s);
    if (kind == kACW)
        return u8 ? launch_strip_class<W, kACW, true>(dist, prm, nb, s)
                  : launch_strip_class<W, kACW, false>(dist, prm, nb, s);
    if (kind == kCW)
        return u8 ? launch_strip_class<W, kCW, true>(dist, prm, nb, s)
                  : launch_strip_class<W, kCW, false>(dist, prm, nb, s);
    if (kind == kCWV)  // no angle term: the L2 sweep of the rgb layout
        return u8 ? launch_strip_class<W, kCWV, true>(kRgb, prm, nb, s)
                  : launch_strip_class<W, kCWV, false>(kRgb, prm, nb, s);
    return hipErrorInvalidValue;
}
hipError_t launch_strip3(int kind, int dist, bool u8, const FwdParams& prm, int nb, hipStream_t s);
hipError_t launch_strip5(int kind, int dist, bool u8, const FwdParams& prm, int nb, hipStream_t s);
hipError_t launch_strip7(int kind, int dist, bool u8, const FwdParams& prm, int nb, hipStream_t s);
hipError_t launch_strip9(int kind, int dist, bool u8, const FwdParams& prm, int nb, hipStream_t s);
template <int W>
static hipError_t launch_strip_extern(int kind, int dist, bool u8, const FwdParams& prm, int nb,
                                      hipStream_t s) {
    if constexpr (W == 3) return launch_strip3(kind, dist, u8, prm, nb, s);
    else if constexpr (W == 5) return launch_strip5(kind, dist, u8, prm, nb, s);
    else if constexpr (W == 7) return launch_strip7(kind, dist, u8, prm, nb, s);
    else return launch_strip9(kind, dist, u8, prm, nb, s);
}

}  // namespace odf
