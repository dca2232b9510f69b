// general.hip -- BVDF and DDF (eqs. 1-3) at the odd windows 11x11, 13x13 and
// 15x15 (Section II: a sqrt(n) x sqrt(n) window of any odd size), ACWDDF and
// the centre-weighted filters of Section III (eq. 9) at 9x9 to 15x15, and the
// hard backward of the selections.
//
// The tile kernels keep a window's n aggregates in registers per thread and
// share pair terms between windows through LDS planes; past 9x9 (81
// aggregates) that no longer fits, so these windows run a direct form: one
// workgroup per 8 x 8 block of windows with the (8 + 2h)^2 pixels they read in
// LDS, one lane per window and one member of it at a time (a wave handles the
// same member u of 64 windows), the member's aggregates summed over the n
// members v in index order with compensated (Kahan) summation, so that a sum of
// up to 225 terms keeps the few-ulp accuracy of the tile kernels' short box
// sums instead of growing with n.  Every pair term of a window is evaluated, the
// member's own pair included, by the same function as for any other pair:
// members of equal colour (and, for BVDF on uint8, of collinear colours, which
// share their canonical direction) then sum identical terms in the same order
// and tie exactly, and the lowest index wins the 64-bit (objective bits,
// index) LDS minimum.  The member index is a byte, which bounds n at 225.
// The centre-weighted kinds keep, beside A and D, the member's terms with the
// window centre (cA, cD), from which the weights of eq. (9) form the levels'
// objectives as in the tile kernels; ACWDDF's switching statistic is then
// taken from the three levels' selections.
#include "aggregates.h"
#include "canon.h"
#include "odf_internal.h"

namespace odf {
namespace {

constexpr int kGenTile = 8;                      // windows per side of a block
constexpr int kGenThreads = 256;                 // 4 waves
constexpr int kGenMaxH = 7;                      // 15 x 15
constexpr int kGenExt = kGenTile + 2 * kGenMaxH;  // 22: pixels per side of a block's read

// Order bits of one member's objective (the same arithmetic as the tile
// kernels' key bits: a non-negative value's bit pattern, or order_key of the
// logarithmic form).
__device__ __forceinline__ uint32_t general_key_bits(int mode, float p, float A, float D) {
    if (mode == kObjA) return __float_as_uint(A);
    if (mode == kObjD) return __float_as_uint(D);
    if (mode == kObjProd) return __float_as_uint(A * D);
    if (mode == kObjQuarter) return __float_as_uint((A * A) * (A * D));
    return order_key(fmaf(1.0f - p, __builtin_amdgcn_logf(A), p * __builtin_amdgcn_logf(D)));
}

template <int KIND, int DIST, bool U8>
__global__ void __launch_bounds__(kGenThreads) fwd_general_kernel(FwdParams prm, int w) {
    constexpr bool CANON = U8 && KIND == kBVDF;  // as in the tile form
    constexpr bool ANG = KIND != kCWV;           // CWVMF^k has no angular term
    constexpr bool L2 = KIND != kBVDF;
    constexpr int NKEY = KIND == kACW ? 4 : 1;    // ACWDDF: eq. (3) and three levels
    constexpr int NWIN = kGenTile * kGenTile;
    __shared__ float4 s_dir[kGenExt * kGenExt];
    __shared__ float4 s_raw[U8 ? 1 : kGenExt * kGenExt];
    __shared__ float s_inv[U8 ? kGenExt * kGenExt : 1];
    __shared__ unsigned long long s_key[NKEY * NWIN];

    const int t = flat_block(prm.grid.n);
    if (t < 0) return;
    const TileCoord tc = tile_coord(xcd_item(t, prm.grid.n), prm.grid);
    const int b = tc.b, ty0 = tc.ty * kGenTile, tx0 = tc.tx * kGenTile;
    const int M = prm.M, N = prm.N;
    const int h = w / 2, n = w * w, E = kGenTile + 2 * h;
    const int tid = threadIdx.x;

    // a1: the block's pixels with their replicated border
    for (int i = tid; i < E * E; i += kGenThreads) {
        const int ey = i / E, ex = i - ey * E;
        const int gy = min(max(ty0 - h + ey, 0), M - 1);
        const int gx = min(max(tx0 - h + ex, 0), N - 1);
        const size_t pix = ((size_t)b * M + gy) * N + gx;
        float4 d, r;
        if constexpr (U8) {
            const uint8_t* s = static_cast<const uint8_t*>(prm.img) + pix * 3;
            const uint32_t c0 = s[0], c1 = s[1], c2 = s[2];
            if constexpr (CANON) {
                float d0, d1, d2;
                canonical_direction(c0, c1, c2, d0, d1, d2);
                prepare_pixel<DIST, true, true>((float)c0, (float)c1, (float)c2, d, r, d0, d1, d2);
            } else {
                prepare_pixel<DIST, true>((float)c0, (float)c1, (float)c2, d, r);
            }
            s_inv[i] = r.w;
        } else {
            const float* s = static_cast<const float*>(prm.img) + pix * 3;
            prepare_pixel<DIST, false>(s[0], s[1], s[2], d, r);
            s_raw[i] = r;
        }
        s_dir[i] = d;
    }
    for (int i = tid; i < NKEY * NWIN; i += kGenThreads) s_key[i] = ~0ull;
    __syncthreads();

    // a2-a4: lane = window (cy, cx) of the block, wave = members u = wave, wave + 4, ...
    const int lane = tid & 63, wave = tid >> 6;
    const int cy = lane / kGenTile, cx = lane % kGenTile;
    const bool in_image = ty0 + cy < M && tx0 + cx < N;
    const int mode = objective_mode<KIND>(prm.p);
    const float p = prm.p;
    const AtanCoef ac = atan_coef();
    for (int u = wave; u < n; u += kGenThreads / 64) {
        const int uy = u / w, ux = u - uy * w;
        const int m = (cy + uy) * E + cx + ux;
        const float4 a = s_dir[m];
        const float ia = s_inv[U8 ? m : 0];  // uint8 images only
        const float4 ra = s_raw[U8 ? 0 : m];  // float images only
        const bool a_zero = U8 && a.w < 0.0f;
        const uint64_t a_zero_wave = U8 ? __builtin_amdgcn_ballot_w64(a_zero) : 0;
        float A = 0.0f, D = 0.0f, kA = 0.0f, kD = 0.0f;  // sums and their compensations
        float tcen = 0.0f, lcen = 0.0f;                   // the terms with the centre
        for (int vy = 0; vy < w; ++vy) {
            const int row = (cy + vy) * E + cx;
            for (int vx = 0; vx < w; ++vx) {
#pragma clang fp contract(off)
                const int v = row + vx;
                float th = 0.0f, l2 = 0.0f;
                if constexpr (U8) {
                    pair_u8<KIND, DIST, ANG, L2>(a, ia, a_zero, a_zero_wave, s_dir[v], s_inv[v],
                                                 prm.coef, ac, th, l2);
                } else {
                    const float4 rb = s_raw[v];
                    if (ANG) th = pair_term<KIND, DIST, false>(a, ra, s_dir[v], rb, prm.coef, ac);
                    if (L2) l2 = l2_term(ra, rb);
                }
                if (ANG) {
                    const float yA = th - kA, tA = A + yA;
                    kA = (tA - A) - yA;
                    A = tA;
                }
                if (L2) {
                    const float yD = l2 - kD, tD = D + yD;
                    kD = (tD - D) - yD;
                    D = tD;
                }
                if (centre_weighted(KIND) && vy == h && vx == h) {
                    tcen = th;
                    lcen = l2;
                }
            }
        }
        const unsigned long long uu = (unsigned)u;
        if (!in_image) continue;
        if constexpr (KIND == kACW) {
            // eq. (3) and the three levels of eq. (9): the centre's weight
            // w_d(k) adds w_d(k) - 1 times the centre term to both sums
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float o = j == 0 ? A * D
                                       : fmaf(prm.acw_wm1[j - 1], tcen, A) *
                                             fmaf(prm.acw_wm1[j - 1], lcen, D);
                atomicMin(&s_key[j * NWIN + lane], ((unsigned long long)__float_as_uint(o) << 32) | uu);
            }
        } else if constexpr (KIND == kCW || KIND == kCWV) {
            const float w1 = prm.acw_wm1[0];
            const float dw = fmaf(w1, lcen, D);
            const float o = KIND == kCWV ? dw : fmaf(w1, tcen, A) * dw;
            atomicMin(&s_key[lane], ((unsigned long long)__float_as_uint(o) << 32) | uu);
        } else {
            const uint32_t bits = general_key_bits(mode, p, A, D);
            atomicMin(&s_key[lane], ((unsigned long long)bits << 32) | uu);
        }
    }
    __syncthreads();

    // the selected member of every in-image window, copied from the image
    if (tid >= NWIN || !in_image) return;
    const int gy = ty0 + cy, gx = tx0 + cx;
    int u = min((int)(s_key[tid] & 0xffu), n - 1);
    if constexpr (KIND == kACW) {
        // switch: S = sum over the three levels of A(y_k, x_d) L2(y_k, x_d); the
        // eq. (3) selection if S > T, else the centre
        const int c = (cy + h) * E + cx + h;
        const float4 cd = s_dir[c];
        float S = 0.0f;
#pragma unroll
        for (int j = 1; j <= 3; ++j) {
            const int uj = min((int)(s_key[j * NWIN + tid] & 0xffu), n - 1);
            const int m = (cy + uj / w) * E + cx + uj % w;
            float th, l2;
            if constexpr (U8) {
                const float4 md = s_dir[m];
                const bool mz = md.w < 0.0f;
                pair_u8<KIND, DIST, true, true>(md, s_inv[m], mz, __builtin_amdgcn_ballot_w64(mz),
                                                cd, s_inv[c], prm.coef, ac, th, l2);
            } else {
                const float4 cr = s_raw[c];
                th = pair_term<KIND, DIST, false>(s_dir[m], s_raw[m], cd, cr, prm.coef, ac);
                l2 = l2_term(s_raw[m], cr);
            }
            S += th * l2;
        }
        if (!(S > prm.acw_T)) u = (n - 1) / 2;
    }
    const int sy = min(max(gy + u / w - h, 0), M - 1);
    const int sx = min(max(gx + u % w - h, 0), N - 1);
    const size_t pix = ((size_t)b * M + gy) * N + gx;
    const size_t src = ((size_t)b * M + sy) * N + sx;
    if constexpr (U8) {
        const uint8_t* s = static_cast<const uint8_t*>(prm.img) + src * 3;
        uint8_t* o = static_cast<uint8_t*>(prm.out) + pix * 3;
        o[0] = s[0]; o[1] = s[1]; o[2] = s[2];
    } else {
        const float* s = static_cast<const float*>(prm.img) + src * 3;
        float* o = static_cast<float*>(prm.out) + pix * 3;
        o[0] = s[0]; o[1] = s[1]; o[2] = s[2];
    }
    if (prm.idx) prm.idx[pix] = (uint8_t)u;
}

template <int KIND, bool U8>
hipError_t launch_general_k(int window, int dist, const FwdParams& prm, hipStream_t s) {
    FwdParams q = prm;
    q.grid = tile_grid(prm.B, (prm.N + kGenTile - 1) / kGenTile,
                       (prm.M + kGenTile - 1) / kGenTile);
    const dim3 grid = flat_grid(q.grid.n), block(kGenThreads);
    if constexpr (KIND == kCWV) {  // no angular term
        (void)dist;
        hipLaunchKernelGGL((fwd_general_kernel<KIND, kRgb, U8>), grid, block, 0, s, q, window);
    } else {
        switch (dist) {
        case kExact:
            hipLaunchKernelGGL((fwd_general_kernel<KIND, kExact, U8>), grid, block, 0, s, q,
                               window);
            break;
        case kMinimax:
            hipLaunchKernelGGL((fwd_general_kernel<KIND, kMinimax, U8>), grid, block, 0, s, q,
                               window);
            break;
        default:
            hipLaunchKernelGGL((fwd_general_kernel<KIND, kRgb, U8>), grid, block, 0, s, q, window);
            break;
        }
    }
    return hipGetLastError();
}

// Hard backward: dx(q) = sum of dy(c) over the windows c that selected a member
// read from q (replicated border); such windows lie within h of q on both axes,
// and they are visited in raster order with the sum in binary64, rounded once
// -- the order and precision of the definition's own accumulation.  Index
// entries >= n route nothing.
__global__ void __launch_bounds__(256) bwd_general_kernel(const uint8_t* __restrict__ idx,
                                                          const float* __restrict__ dy,
                                                          float* __restrict__ dx, int M, int N,
                                                          TileGrid tg, int w) {
    const int t = flat_block(tg.n);
    if (t < 0) return;
    const TileCoord tc = tile_coord(t, tg);  // 64 x 4 pixels per workgroup
    const int qx = tc.tx * 64 + (threadIdx.x & 63), qy = tc.ty * 4 + (threadIdx.x >> 6);
    if (qx >= N || qy >= M) return;
    const int h = w / 2, n = w * w;
    const size_t base = (size_t)tc.b * M * N;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int cy = max(qy - h, 0); cy <= min(qy + h, M - 1); ++cy) {
        for (int cx = max(qx - h, 0); cx <= min(qx + h, N - 1); ++cx) {
            const size_t c = base + (size_t)cy * N + cx;
            const int u = idx[c];
            if (u >= n) continue;
            const int sy = min(max(cy + u / w - h, 0), M - 1);
            const int sx = min(max(cx + u % w - h, 0), N - 1);
            if (sy != qy || sx != qx) continue;
            a0 += (double)dy[3 * c + 0];
            a1 += (double)dy[3 * c + 1];
            a2 += (double)dy[3 * c + 2];
        }
    }
    float* o = dx + (base + (size_t)qy * N + qx) * 3;
    o[0] = (float)a0;
    o[1] = (float)a1;
    o[2] = (float)a2;
}

}  // namespace

hipError_t launch_forward_general(int window, int kind, int dist, bool u8, const FwdParams& prm,
                                  hipStream_t s) {
    // BVDF / DDF from 11x11 (9x9 and below run the tiles), the centre-weighted
    // kinds from 9x9
    const int lo = centre_weighted(kind) ? 9 : 11;
    if (window < lo || window > 2 * kGenMaxH + 1 || window % 2 == 0) return hipErrorInvalidValue;
    switch (kind) {
    case kBVDF:
        return u8 ? launch_general_k<kBVDF, true>(window, dist, prm, s)
                  : launch_general_k<kBVDF, false>(window, dist, prm, s);
    case kDDF:
        return u8 ? launch_general_k<kDDF, true>(window, dist, prm, s)
                  : launch_general_k<kDDF, false>(window, dist, prm, s);
    case kACW:
        return u8 ? launch_general_k<kACW, true>(window, dist, prm, s)
                  : launch_general_k<kACW, false>(window, dist, prm, s);
    case kCW:
        return u8 ? launch_general_k<kCW, true>(window, dist, prm, s)
                  : launch_general_k<kCW, false>(window, dist, prm, s);
    case kCWV:  // no angular term: one form for every dist
        return u8 ? launch_general_k<kCWV, true>(window, dist, prm, s)
                  : launch_general_k<kCWV, false>(window, dist, prm, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_backward_hard_general(int window, const uint8_t* idx, const float* dy, float* dx,
                                        int B, int M, int N, hipStream_t s) {
    if (window < 3 || window > 2 * kGenMaxH + 1 || window % 2 == 0) return hipErrorInvalidValue;
    const TileGrid tg = tile_grid(B, (N + 63) / 64, (M + 3) / 4);
    hipLaunchKernelGGL(bwd_general_kernel, flat_grid(tg.n), dim3(256), 0, s, idx, dy, dx, M, N,
                       tg, window);
    return hipGetLastError();
}

}  // namespace odf
