// softmin.hip -- temperature-tau softmin relaxation of the argmin and its
// gradient (float32 images, exact angle of eq. 2, DDF objective
// Omega = A^(1-p) D^p or BVDF Omega = A).
//
// Forward, per window c:  pi_u = exp(-(Omega_u - min Omega) / tau) / Z,
//                         y(c) = sum_u pi_u x(c + u).
// Backward (reverse mode of the same expression, written for the tile):
//   direct term      dx(q) += pi_u(c) dy(c)                   (q = c + u)
//   through Omega    g_u(c) = -pi_u (x_u - y(c)) . dy(c) / tau,
//                    G^A_u(c) = g_u dOmega/dA_u, G^D_u(c) = g_u dOmega/dD_u
//   through the pair terms: with A_u(c) = sum_v theta(x_{c+u}, x_{c+v}),
//     dx(q) += sum_{r != q} S(q, r) grad_1 theta(q, r),
//     S(q, r) = sum over windows c containing q and r of G_{u_q}(c) + G_{u_r}(c)
//             = B_q(r - q) + B_r(q - r),
//     B_p(d) = sum of G_u(p - u) over the members u of windows that contain
//              both p and p + d (a box sum of the transposed window grid);
//   the same for D with the L2 gradient.
// Each workgroup handles the windows of its tile and produces gradient
// contributions for every pixel of its extended tile; contributions of
// replicated border positions are folded into their source pixel inside the
// tile, written per tile to a workspace, and summed over the (at most four)
// overlapping tiles by a second kernel in a fixed order, so the result does
// not depend on scheduling.
#include "aggregates.h"
#include "odf_internal.h"

namespace odf {

// Extended tile of the softmin kernels (one thread per extended pixel).  The
// 5x5 forward parks the angle part of every objective in LDS between its two
// sweeps, which frees the registers for 1024-thread tiles.  The backward uses
// 512-thread tiles; it parks the angle sums A during the L2 sweep as well and
// recomputes Omega from A and D where it needs it, so that (with 128 VGPRs) two
// workgroups share a compute unit.  7x7 and 9x9 keep 512-thread tiles both ways
// (26 x 10 and 24 x 8 windows): their 49 or 81 weights per window fill 77-114 KB
// of LDS, one workgroup per compute unit, so the backward may take 256 VGPRs
// for its two sets of member aggregates (9x9 spills part of them).
template <int W, int KIND, bool BWD>
struct SoftTile {
    static constexpr int EXT_W = 32;
    static constexpr int EXT_H = (W == 5 && !BWD) ? 32 : 16;
    static constexpr int NT = EXT_W * EXT_H;
};

template <int W, bool BWD>
constexpr int soft_waves_per_eu() {
    if (!BWD) return 1;
    return W >= 7 ? 2 : 4;
}

__device__ __forceinline__ float key_value(uint32_t k) {
    uint32_t bits = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(bits);
}

// The hardware base-2 logarithm and power (about 1 ulp; the aggregates are 0 or
// normal numbers, and log2(0) = -inf gives the power 0 as it should).
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// The objective A^(1-p) D^p (BVDF: A) from the hardware log2 / exp2.
template <int KIND>
__device__ __forceinline__ float soft_objective(float A, float D, float p) {
    if (KIND == kBVDF || p == 0.0f) return A;
    if (p == 1.0f) return D;
    return hw_exp2(fmaf(1.0f - p, hw_log2(A), p * hw_log2(D)));
}

// dOmega/dA and dOmega/dD (0 where a fractional power meets a zero aggregate),
// with the hardware reciprocal (about 1 ulp).
template <int KIND>
__device__ __forceinline__ void objective_grad(float A, float D, float Om, float p, float& dA,
                                               float& dD) {
    if (KIND == kBVDF || p == 0.0f) { dA = 1.0f; dD = 0.0f; return; }
    if (p == 1.0f) { dA = 0.0f; dD = 1.0f; return; }
    dA = A > 0.0f ? ((1.0f - p) * Om) * __builtin_amdgcn_rcpf(A) : 0.0f;
    dD = D > 0.0f ? (p * Om) * __builtin_amdgcn_rcpf(D) : 0.0f;
}

// u*v - w*z to within a rounding of the exact value: the rounding error of
// w*z is recovered with a fused multiply-add (Dekker's two-product).
__device__ __forceinline__ float cross_term(float u, float v, float w, float z) {
    const float p = w * z;
    const float e = fmaf(w, z, -p);
    return fmaf(u, v, -p) - e;
}

// grad_1 theta(a, b) = (a x c) / (|c| |a|^2) with c = a x b, on the directions a,
// b of the two pixels, times da/dx for the raw first pixel.  It is linear in
// c / |c|: the gradient of a member over all its neighbours r, sum_r S_r
// grad_1 theta(a, r), is a x (sum_r S_r c_r / |c_r|) / |a|^2, so the neighbour
// loop accumulates S_r c_r / |c_r| and the cross product with the member's own
// direction is taken once.  c is formed to full relative accuracy (a
// two-product difference per component) and a x c is well conditioned (c is
// orthogonal to a), so nearly parallel pairs keep an accurate gradient
// direction; equal directions give c = 0 exactly and contribute nothing.
__device__ __forceinline__ void add_cross_dir(const float4& a, const float4& b, float S, float& v0,
                                              float& v1, float& v2) {
    const float c0 = cross_term(a.y, b.z, a.z, b.y);
    const float c1 = cross_term(a.z, b.x, a.x, b.z);
    const float c2 = cross_term(a.x, b.y, a.y, b.x);
    const float s2 = fmaf(c0, c0, fmaf(c1, c1, c2 * c2));
    const float w = s2 > 0.0f ? S * rsq(s2) : 0.0f;
    v0 = fmaf(w, c0, v0);
    v1 = fmaf(w, c1, v1);
    v2 = fmaf(w, c2, v2);
}

// S grad_1 |a - b| = S (a - b) / |a - b| (0 for a = b), accumulated.
__device__ __forceinline__ void add_l2_dir(const float4& a, const float4& b, float S, float& v0,
                                           float& v1, float& v2) {
    const float e0 = a.x - b.x, e1 = a.y - b.y, e2 = a.z - b.z;
    const float l2 = fmaf(e0, e0, fmaf(e1, e1, e2 * e2));
    const float w = l2 > 0.0f ? S * rsq(l2) : 0.0f;
    v0 = fmaf(w, e0, v0);
    v1 = fmaf(w, e1, v1);
    v2 = fmaf(w, e2, v2);
}

// 2D prefix sums of the member gradients gr (row-major w x w):
// P[i][j] = sum of gr over rows < i and columns < j.
template <int W>
__device__ __forceinline__ void member_prefix(const float (&gr)[W * W], float (&P)[W + 1][W + 1]) {
#pragma unroll
    for (int j = 0; j <= W; ++j) P[0][j] = 0.0f;
#pragma unroll
    for (int y = 0; y < W; ++y) {
        P[y + 1][0] = 0.0f;
        float row = 0.0f;
#pragma unroll
        for (int x = 0; x < W; ++x) {
            row += gr[y * W + x];
            P[y + 1][x + 1] = P[y][x + 1] + row;
        }
    }
}

// Sum of gr[u] over the members u = (uy, ux) of windows containing both p and
// p + d: the rectangle uy in [max(-h, -h - dy), min(h, h - dy)] (and likewise
// for ux), read from the prefix table (d is a compile-time offset).
template <int W>
__device__ __forceinline__ float box_over_members(const float (&P)[W + 1][W + 1], int dy, int dx) {
    constexpr int H = W / 2;
    const int y0 = dy < 0 ? -dy : 0, y1 = dy > 0 ? 2 * H - dy : 2 * H;
    const int x0 = dx < 0 ? -dx : 0, x1 = dx > 0 ? 2 * H - dx : 2 * H;
    return (P[y1 + 1][x1 + 1] - P[y0][x1 + 1]) - (P[y1 + 1][x0] - P[y0][x0]);
}

// Offsets of the gradient exchange, the forward half of the pair offsets
// (delta > 0 in row-major order: row g = 0 with dx > 0, rows g > 0 with any
// dx), in chunks of at most 2h + 1 offsets of one row: g = 0 takes dx = 1..2h,
// every g > 0 takes dx = -2h..0 and then dx = 1..2h.
template <int W>
struct PairChunks {
    static constexpr int H = W / 2, N = 1 + 2 * (2 * H), CMAX = 2 * H + 1;
    static constexpr int g(int k) { return (k + 1) / 2; }
    static constexpr int lo(int k) { return (k % 2 == 0) ? 1 : -2 * H; }
    static constexpr int hi(int k) { return (k % 2 == 0) ? 2 * H : 0; }
};

// Pair-term part of the gradient for one plane (angle, or L2 when L2PASS):
// dx(q) += sum_{r != q} S(q, r) grad_1 term(q, r), S(q, r) = B_q(r - q) +
// B_r(q - r) (symmetric).  Each unordered pair is evaluated once, by its first
// pixel q (r = q + delta, delta in the forward half).  Accumulated as
// S c / |c| (angle, c = d_q x d_r, crossed with the member's own direction at
// the end) or S e / |e| (L2, e = x_q - x_r), the second pixel's share is the
// same vector negated (c and e change sign with the order of the pair, S and
// |c|, |e| do not), so q adds it and hands it to r through LDS.  Per chunk of
// offsets: every pixel publishes B(-delta) (plane P), then q forms S and the
// pair's share (plane Q, three floats), then r subtracts the shares meant for
// it -- all in a fixed order, so the result is deterministic.
// scale: da/dx / |a|^2 of this member's direction (angle plane only).
template <int W, int EXT_W, int EXT_H, bool L2PASS>
__device__ __forceinline__ void propagate_pairs(const float (&gr)[W * W],
                                                const float4* __restrict__ s_dir,
                                                const float4* __restrict__ s_raw,
                                                float* __restrict__ s_plane, int ey, int ex,
                                                int tid, const float4& mdir, const float4& mraw,
                                                float scale, float& gx0, float& gx1, float& gx2) {
    using Ch = PairChunks<W>;
    constexpr int NT = EXT_W * EXT_H, CMAX = Ch::CMAX;
    float* P = s_plane;                // [CMAX][NT]: B_r(-delta) of the chunk's offsets
    float* Q = s_plane + CMAX * NT;    // [3][CMAX][NT]: the share handed to r = q + delta
    float Pt[W + 1][W + 1];
    member_prefix<W>(gr, Pt);
    float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f;
    auto receive = [&](int k) {        // the shares of chunk k meant for this pixel
        const int g = Ch::g(k);
#pragma unroll
        for (int dx = Ch::lo(k); dx <= Ch::hi(k); ++dx) {
            const int qy = ey - g, qx = ex - dx;  // q = this pixel - delta
            if (qy < 0 || qx < 0 || qx >= EXT_W) continue;
            const int j = (dx - Ch::lo(k)) * NT + qy * EXT_W + qx;
            v0 -= Q[j];
            v1 -= Q[CMAX * NT + j];
            v2 -= Q[2 * CMAX * NT + j];
        }
    };
#pragma unroll
    for (int k = 0; k < Ch::N; ++k) {
        const int g = Ch::g(k);
#pragma unroll
        for (int dx = Ch::lo(k); dx <= Ch::hi(k); ++dx)
            P[(dx - Ch::lo(k)) * NT + tid] = box_over_members<W>(Pt, -g, -dx);
        if (k > 0) receive(k - 1);
        __syncthreads();
#pragma unroll
        for (int dx = Ch::lo(k); dx <= Ch::hi(k); ++dx) {
            const int ry = ey + g, rx = ex + dx;
            if (ry >= EXT_H || rx < 0 || rx >= EXT_W) continue;
            const int r = ry * EXT_W + rx;
            const float S = box_over_members<W>(Pt, g, dx) + P[(dx - Ch::lo(k)) * NT + r];
            float w0 = 0.0f, w1 = 0.0f, w2 = 0.0f;
            if (L2PASS) add_l2_dir(mraw, s_raw[r], S, w0, w1, w2);
            else add_cross_dir(mdir, s_dir[r], S, w0, w1, w2);
            v0 += w0;
            v1 += w1;
            v2 += w2;
            const int j = (dx - Ch::lo(k)) * NT + tid;
            Q[j] = w0;
            Q[CMAX * NT + j] = w1;
            Q[2 * CMAX * NT + j] = w2;
        }
        __syncthreads();
    }
    receive(Ch::N - 1);
    if (L2PASS) {
        gx0 += v0;
        gx1 += v1;
        gx2 += v2;
    } else {
        // a x (sum S c / |c|), times da/dx / |a|^2
        gx0 = fmaf(fmaf(mdir.y, v2, -mdir.z * v1), scale, gx0);
        gx1 = fmaf(fmaf(mdir.z, v0, -mdir.x * v2), scale, gx1);
        gx2 = fmaf(fmaf(mdir.x, v1, -mdir.y * v0), scale, gx2);
    }
}

template <int W, int KIND, bool BWD>
__global__ void __launch_bounds__((SoftTile<W, KIND, BWD>::NT))
    __attribute__((amdgpu_waves_per_eu(soft_waves_per_eu<W, BWD>()))) softmin_kernel(SoftParams prm) {
    constexpr int EXT_W = SoftTile<W, KIND, BWD>::EXT_W, EXT_H = SoftTile<W, KIND, BWD>::EXT_H;
    using Gm = FwdGeom<W, EXT_W, EXT_H>;
    constexpr int H = Gm::H, NW = Gm::NW, G = Gm::G, TW = Gm::TW, TH = Gm::TH, NT = Gm::NT;
    constexpr int TT = TW * TH;
    // planes: G for the aggregate sweeps; the gradient exchange takes 4 CMAX
    // (plane P and the three planes of Q)
    constexpr int NPLANE =
        BWD && 4 * PairChunks<W>::CMAX > G ? 4 * PairChunks<W>::CMAX : G;

    // LDS: the pixels, the window keys and one region that holds, in turn, the
    // planes of the aggregate sweeps, the (member, window) weights e with the
    // per-window sums, and (backward) the planes of the gradient propagation.  The
    // forward-only kernel keeps the angle part of each objective in e during its
    // L2 sweep, so there e follows the planes instead of sharing their space; the
    // DDF backward parks A in the same place during its L2 sweep.
    constexpr int NE = NW * TT, NWIN = BWD ? 8 * TT : 0;
    constexpr int R0 = NPLANE * NT > NE + NWIN ? NPLANE * NT : NE + NWIN;
    constexpr int RP = KIND == kDDF ? G * NT + NE : 0;  // planes + parked angle sums
    constexpr int REGION = BWD ? (R0 > RP ? R0 : RP) : G * NT + NE;
    // One struct, in this order, so that the unguarded aggregate sweeps
    // (aggregates.h) read past the pixel arrays and before the planes inside it.
    struct Lds {
        float4 dir[NT];
        float4 raw[NT];
        uint32_t key[TT];
        float buf[REGION];
    };
    __shared__ Lds sh;
    constexpr size_t kOver = 2 * H * EXT_W + 2 * H;
    static_assert(offsetof(Lds, dir) + (NT + kOver) * sizeof(float4) <= sizeof(Lds), "dir");
    static_assert(offsetof(Lds, raw) + (NT + kOver) * sizeof(float4) <= sizeof(Lds), "raw");
    static_assert(offsetof(Lds, buf) >= kOver * sizeof(float), "planes");
    float4* const s_dir = sh.dir;
    float4* const s_raw = sh.raw;
    uint32_t* const s_key = sh.key;
    float* const s_buf = sh.buf;
    float* const s_plane = s_buf;
    float* const s_e = BWD ? s_buf : s_buf + G * NT;
    float* const s_win = s_e + NE;  // backward only

    const int tid = threadIdx.x;
    const int ey = tid / EXT_W, ex = tid - ey * EXT_W;
    const int tile = flat_block(prm.grid.n);
    if (tile < 0) return;
    const TileCoord tc = tile_coord(tile, prm.grid);
    const int b = tc.b;
    const int ty0 = tc.ty * TH, tx0 = tc.tx * TW;
    const int M = prm.M, N = prm.N;
    const float p = prm.p;
    const float inv_tau = prm.inv_tau;
    const float tau_ln2 = 0.69314718055994531f / inv_tau;  // tau ln 2: ln e = ln2 log2 e

    {
        const int gy = min(max(ty0 - H + ey, 0), M - 1);
        const int gx = min(max(tx0 - H + ex, 0), N - 1);
        const float* s = prm.x + (((size_t)b * M + gy) * N + gx) * 3;
        float4 d, r;
        prepare_pixel<kExact, false>(s[0], s[1], s[2], d, r);
        s_dir[tid] = d;
        s_raw[tid] = r;
    }
    for (int i = tid; i < TT; i += NT) s_key[i] = 0xffffffffu;
    __syncthreads();
    const float4 mdir = s_dir[tid];
    const float4 mraw = s_raw[tid];
    const MinimaxCoef no_coef{};

    // Bit k of `rows` (`cols`): the window k rows above (columns left of) this
    // extended position is an in-image window of the output tile.  Member u of the
    // window c lies here iff both bits of u's row and column are set.
    uint32_t rows = 0, cols = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int cy = ey - k, cx = ex - k;
        if (cy >= 0 && cy < TH && ty0 + cy < M) rows |= 1u << k;
        if (cx >= 0 && cx < TW && tx0 + cx < N) cols |= 1u << k;
    }
    const int cbase = ey * TW + ex;
    auto window_of = [&](int u, int& c) -> bool {
        c = cbase - (u / W) * TW - u % W;
        return ((rows >> (u / W)) & (cols >> (u % W)) & 1u) != 0;
    };

    float A[NW], D[NW];
    const TilePix px{s_dir, s_raw, nullptr};
    // unguarded sweeps: only windows of the output tile (window_of) are used below
    member_aggregates<W, KIND, kExact, false, EXT_W, EXT_H, false, false>(
        px, s_plane, ey, ex, tid, mdir, mraw, no_coef, A);
    if constexpr (!BWD) {
        // forward only: the angle part of each objective waits in s_e (same
        // (member, window) layout) during the L2 sweep; then s_e holds Omega
        const int mode = (KIND == kBVDF || p == 0.0f) ? 0 : (p == 1.0f ? 1 : 2);
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            int c;
            if (window_of(u, c)) s_e[u * TT + c] = mode == 2 ? (1.0f - p) * hw_log2(A[u]) : A[u];
        }
        if (KIND == kDDF)
            member_aggregates<W, KIND, kExact, false, EXT_W, EXT_H, true, false>(
                px, s_plane, ey, ex, tid, mdir, mraw, no_coef, D);
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            int c;
            if (!window_of(u, c)) continue;
            const float part = s_e[u * TT + c];
            const float om = mode == 0 ? part
                                       : (mode == 1 ? D[u] : hw_exp2(fmaf(p, hw_log2(D[u]), part)));
            s_e[u * TT + c] = om;
            atomicMin(&s_key[c], order_key(om));
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            int c;
            if (window_of(u, c))
                s_e[u * TT + c] = __expf((key_value(s_key[c]) - s_e[u * TT + c]) * inv_tau);
        }
    } else {
        if (KIND == kDDF) {
            float* const s_park = s_buf + G * NT;
#pragma unroll
            for (int u = 0; u < NW; ++u) {
                int c;
                if (window_of(u, c)) s_park[u * TT + c] = A[u];
            }
            member_aggregates<W, KIND, kExact, false, EXT_W, EXT_H, true, false>(
                px, s_plane, ey, ex, tid, mdir, mraw, no_coef, D);
#pragma unroll
            for (int u = 0; u < NW; ++u) {
                int c;
                A[u] = window_of(u, c) ? s_park[u * TT + c] : 0.0f;
            }
        } else {
#pragma unroll
            for (int u = 0; u < NW; ++u) D[u] = 0.0f;
        }
        // Omega once per (member, window): kept in e for the minimum, then
        // replaced there by the weight
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            int c;
            if (window_of(u, c)) {
                const float om = soft_objective<KIND>(A[u], D[u], p);
                s_e[u * TT + c] = om;
                atomicMin(&s_key[c], order_key(om));
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            int c;
            if (window_of(u, c))
                s_e[u * TT + c] = __expf((key_value(s_key[c]) - s_e[u * TT + c]) * inv_tau);
        }
    }
    __syncthreads();

    // per window: Z, y (and dy for the backward), members in index order
    for (int i = tid; i < TT; i += NT) {
        const int cy = i / TW, cx = i - (i / TW) * TW;
        const int gy = ty0 + cy, gx = tx0 + cx;
        if (gy >= M || gx >= N) continue;
        float z = 0.0f;
#pragma unroll
        for (int u = 0; u < NW; ++u) z += s_e[u * TT + i];
        const float iz = 1.0f / z;
        float y0 = 0.0f, y1 = 0.0f, y2 = 0.0f;
#pragma unroll
        for (int u = 0; u < NW; ++u) {
            const float pi = s_e[u * TT + i] * iz;
            const float4 r = s_raw[(cy + u / W) * EXT_W + cx + u % W];
            y0 = fmaf(pi, r.x, y0);
            y1 = fmaf(pi, r.y, y1);
            y2 = fmaf(pi, r.z, y2);
        }
        const size_t pix = ((size_t)b * M + gy) * N + gx;
        if (!BWD) {
            prm.y[pix * 3 + 0] = y0;
            prm.y[pix * 3 + 1] = y1;
            prm.y[pix * 3 + 2] = y2;
        } else {
            float* w = s_win + 8 * i;
            w[0] = iz; w[1] = y0; w[2] = y1; w[3] = y2;
            w[4] = prm.dy[pix * 3 + 0];
            w[5] = prm.dy[pix * 3 + 1];
            w[6] = prm.dy[pix * 3 + 2];
        }
    }
    if (!BWD) return;
    __syncthreads();

    // ---------------------------------------------------------------- backward
    float gx0 = 0.0f, gx1 = 0.0f, gx2 = 0.0f;  // dL/dx of this extended position
    // A[] <- G^A, D[] <- G^D (per member u of the window p - u)
#pragma unroll
    for (int u = 0; u < NW; ++u) {
        int c;
        float ga = 0.0f, gd = 0.0f;
        if (window_of(u, c)) {
            const float* w = s_win + 8 * c;
            const float pi = s_e[u * TT + c] * w[0];
            gx0 = fmaf(pi, w[4], gx0);
            gx1 = fmaf(pi, w[5], gx1);
            gx2 = fmaf(pi, w[6], gx2);
            const float t = fmaf(mraw.x - w[1], w[4], fmaf(mraw.y - w[2], w[5], (mraw.z - w[3]) * w[6]));
            const float gom = -pi * t * inv_tau;
            float dA, dD;
            if (KIND == kBVDF || p == 0.0f || p == 1.0f) {
                objective_grad<KIND>(A[u], D[u], 0.0f, p, dA, dD);  // constant derivatives
            } else {
                // Omega from its weight, e = exp((min - Omega) / tau): Omega = min - tau ln e,
                // within a few ulp of tau of the objective (a member with e = 0 has pi = 0
                // and no gradient)
                const float e = s_e[u * TT + c];
                const float om = fmaf(-tau_ln2, __builtin_amdgcn_logf(e), key_value(s_key[c]));
                objective_grad<KIND>(A[u], D[u], e > 0.0f ? om : 0.0f, p, dA, dD);
            }
            ga = gom * dA;
            gd = gom * dD;
        }
        A[u] = ga;
        D[u] = gd;
    }
    // da/dx / |a|^2 for the direction a = 2^-e x (0 for the zero pixel)
    const float scale =
        mraw.w / fmaf(mdir.x, mdir.x, fmaf(mdir.y, mdir.y, mdir.z * mdir.z));
    __syncthreads();  // every thread is done with e and the window sums: the planes reuse them
    propagate_pairs<W, EXT_W, EXT_H, false>(A, s_dir, s_raw, s_plane, ey, ex, tid, mdir, mraw,
                                            scale, gx0, gx1, gx2);
    if (KIND == kDDF)
        propagate_pairs<W, EXT_W, EXT_H, true>(D, s_dir, s_raw, s_plane, ey, ex, tid, mdir, mraw,
                                               0.0f, gx0, gx1, gx2);

    // fold replicated border positions into their source pixel, then write
    // this tile's contribution for every in-image extended position
    float* s_dx = s_plane;
    s_dx[tid * 3 + 0] = gx0;
    s_dx[tid * 3 + 1] = gx1;
    s_dx[tid * 3 + 2] = gx2;
    __syncthreads();
    const int gy = ty0 - H + ey, gxp = tx0 - H + ex;
    if (gy < 0 || gy >= M || gxp < 0 || gxp >= N) return;
    int eylo = ey, eyhi = ey, exlo = ex, exhi = ex;
    if (gy == 0) eylo = 0;                        // rows above the image clamp to row 0
    if (gy == M - 1) eyhi = EXT_H - 1;            // rows below clamp to row M - 1
    if (gxp == 0) exlo = 0;
    if (gxp == N - 1) exhi = EXT_W - 1;
    float f0 = 0.0f, f1 = 0.0f, f2 = 0.0f;
    for (int yy = eylo; yy <= eyhi; ++yy) {
        const int gyy = min(max(ty0 - H + yy, 0), M - 1);
        if (gyy != gy) continue;
        for (int xx = exlo; xx <= exhi; ++xx) {
            const int gxx = min(max(tx0 - H + xx, 0), N - 1);
            if (gxx != gxp) continue;
            const float* v = s_dx + (yy * EXT_W + xx) * 3;
            f0 += v[0];
            f1 += v[1];
            f2 += v[2];
        }
    }
    float* o = prm.ws + ((size_t)tile * NT + tid) * 3;
    o[0] = f0;
    o[1] = f1;
    o[2] = f2;
}

// dx(q) = sum of the tile contributions at q over the tiles whose extended
// region contains q, in increasing tile order.
template <int W, int KIND>
__global__ void __launch_bounds__(256) softmin_combine(SoftParams prm) {
    constexpr int EXT_W = SoftTile<W, KIND, true>::EXT_W, EXT_H = SoftTile<W, KIND, true>::EXT_H;
    using Gm = FwdGeom<W, EXT_W, EXT_H>;
    constexpr int H = Gm::H, TW = Gm::TW, TH = Gm::TH, NT = Gm::NT;
    const int tiles_x = prm.tiles_x, tiles_y = prm.tiles_y;
    // a 64 x 4 block of output pixels per workgroup
    const int blk = flat_block(prm.cgrid.n);
    if (blk < 0) return;
    const TileCoord bc = tile_coord(blk, prm.cgrid);
    const int gx = bc.tx * 64 + (threadIdx.x & 63);
    const int gy = bc.ty * 4 + (threadIdx.x >> 6);
    const int b = bc.b;
    if (gx >= prm.N || gy >= prm.M) return;
    const int tylo = max(0, (gy - H - TH + 1 + TH * 4) / TH - 4);
    const int tyhi = min(tiles_y - 1, (gy + H) / TH);
    const int txlo = max(0, (gx - H - TW + 1 + TW * 4) / TW - 4);
    const int txhi = min(tiles_x - 1, (gx + H) / TW);
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
    for (int ty = tylo; ty <= tyhi; ++ty) {
        const int ey = gy - (ty * TH - H);
        if (ey < 0 || ey >= EXT_H) continue;
        for (int tx = txlo; tx <= txhi; ++tx) {
            const int ex = gx - (tx * TW - H);
            if (ex < 0 || ex >= EXT_W) continue;
            const size_t tile = ((size_t)b * tiles_y + ty) * tiles_x + tx;
            const float* v = prm.ws + (tile * NT + ey * EXT_W + ex) * 3;
            a0 += v[0];
            a1 += v[1];
            a2 += v[2];
        }
    }
    float* o = prm.dx + (((size_t)b * prm.M + gy) * prm.N + gx) * 3;
    o[0] = a0;
    o[1] = a1;
    o[2] = a2;
}

// Direct form for the odd windows 11 to 15 (the tiles' (member, window) weight
// arrays outgrow the LDS there): one thread per window, every pair term of the
// window evaluated from its definition (n^2 per window, no reuse).  The forward
// forms A, D, Omega and the weights as above; the backward then forms, for
// every member u of its window, pi_u dy + sum_v (G^A_u + G^A_v) grad_1 theta(u, v)
// + (G^D_u + G^D_v) grad_1 |u - v| (the dependence of A_u and of every A_v on
// x_u), written to the workspace (n x 3 floats per pixel), and a gather pass
// sums, for every pixel q, the member gradients read from q over the windows
// within h of q in raster order and their members in index order:
// deterministic.  Per-window arrays live in scratch (n <= 225).
constexpr int kSoftDirMaxN = 225;
constexpr int kSoftDirThreads = 128;

__device__ __forceinline__ void soft_dir_member(const SoftParams& prm, int b, int r, int c, int u,
                                                int w, float4& d, float4& raw) {
    const int h = w / 2;
    const int gy = min(max(r + u / w - h, 0), prm.M - 1);
    const int gx = min(max(c + u % w - h, 0), prm.N - 1);
    const float* s = prm.x + (((size_t)b * prm.M + gy) * prm.N + gx) * 3;
    prepare_pixel<kExact, false>(s[0], s[1], s[2], d, raw);
}

template <int KIND, bool BWD>
__global__ void __launch_bounds__(kSoftDirThreads) softmin_direct_kernel(SoftParams prm, int w) {
    const int blk = flat_block(prm.grid.n);
    if (blk < 0) return;
    const long long mn = (long long)prm.M * prm.N, npix = mn * prm.B;
    const long long pix = (long long)blk * kSoftDirThreads + threadIdx.x;
    if (pix >= npix) return;
    const int b = (int)(pix / mn);
    const int rc = (int)(pix - (long long)b * mn);
    const int r = rc / prm.N, c = rc - r * prm.N;
    const int n = w * w;
    const float p = prm.p, inv_tau = prm.inv_tau;
    const MinimaxCoef no_coef{};
    const AtanCoef ac = atan_coef();
    float A[kSoftDirMaxN], D[kSoftDirMaxN], E[kSoftDirMaxN];
    float omin = __builtin_huge_valf();
    for (int u = 0; u < n; ++u) {
        float4 du, ru;
        soft_dir_member(prm, b, r, c, u, w, du, ru);
        float a = 0.0f, d = 0.0f;
        for (int v = 0; v < n; ++v) {
            float4 dv, rv;
            soft_dir_member(prm, b, r, c, v, w, dv, rv);
            a += pair_term<KIND, kExact, false>(du, ru, dv, rv, no_coef, ac);
            if (KIND == kDDF) d += l2_term(ru, rv);
        }
        A[u] = a;
        D[u] = d;
        E[u] = soft_objective<KIND>(a, d, p);
        omin = fminf(omin, E[u]);
    }
    float z = 0.0f;
    for (int u = 0; u < n; ++u) {
        E[u] = __expf((omin - E[u]) * inv_tau);
        z += E[u];
    }
    const float iz = 1.0f / z;
    float y0 = 0.0f, y1 = 0.0f, y2 = 0.0f;
    for (int u = 0; u < n; ++u) {
        float4 du, ru;
        soft_dir_member(prm, b, r, c, u, w, du, ru);
        const float pu = E[u] * iz;
        y0 = fmaf(pu, ru.x, y0);
        y1 = fmaf(pu, ru.y, y1);
        y2 = fmaf(pu, ru.z, y2);
    }
    if (!BWD) {
        prm.y[pix * 3 + 0] = y0;
        prm.y[pix * 3 + 1] = y1;
        prm.y[pix * 3 + 2] = y2;
        return;
    }
    const float g0 = prm.dy[pix * 3 + 0], g1 = prm.dy[pix * 3 + 1], g2 = prm.dy[pix * 3 + 2];
    // A[], D[] <- G^A, G^D of every member
    for (int u = 0; u < n; ++u) {
        float4 du, ru;
        soft_dir_member(prm, b, r, c, u, w, du, ru);
        const float pu = E[u] * iz;
        const float t = fmaf(ru.x - y0, g0, fmaf(ru.y - y1, g1, (ru.z - y2) * g2));
        const float gom = -pu * t * inv_tau;
        float dA, dD;
        objective_grad<KIND>(A[u], D[u], soft_objective<KIND>(A[u], D[u], p), p, dA, dD);
        A[u] = gom * dA;
        D[u] = gom * dD;
    }
    for (int u = 0; u < n; ++u) {
        float4 du, ru;
        soft_dir_member(prm, b, r, c, u, w, du, ru);
        float v0 = 0.0f, v1 = 0.0f, v2 = 0.0f, l0 = 0.0f, l1 = 0.0f, l2 = 0.0f;
        for (int v = 0; v < n; ++v) {
            float4 dv, rv;
            soft_dir_member(prm, b, r, c, v, w, dv, rv);
            add_cross_dir(du, dv, A[u] + A[v], v0, v1, v2);
            if (KIND == kDDF) add_l2_dir(ru, rv, D[u] + D[v], l0, l1, l2);
        }
        // a x (sum S c / |c|), times da/dx / |a|^2 (0 for the zero pixel)
        const float scale = ru.w / fmaf(du.x, du.x, fmaf(du.y, du.y, du.z * du.z));
        const float pu = E[u] * iz;
        float* o = prm.ws + ((size_t)pix * n + u) * 3;
        o[0] = fmaf(pu, g0, fmaf(fmaf(du.y, v2, -du.z * v1), scale, l0));
        o[1] = fmaf(pu, g1, fmaf(fmaf(du.z, v0, -du.x * v2), scale, l1));
        o[2] = fmaf(pu, g2, fmaf(fmaf(du.x, v1, -du.y * v0), scale, l2));
    }
}

// dx(q): the member gradients of the windows within h of q (raster order)
// whose member u is read from q (replicated border), members in index order.
__global__ void __launch_bounds__(kSoftDirThreads) softmin_direct_gather(SoftParams prm, int w) {
    const int blk = flat_block(prm.grid.n);
    if (blk < 0) return;
    const long long mn = (long long)prm.M * prm.N, npix = mn * prm.B;
    const long long pix = (long long)blk * kSoftDirThreads + threadIdx.x;
    if (pix >= npix) return;
    const int b = (int)(pix / mn);
    const int rc = (int)(pix - (long long)b * mn);
    const int qy = rc / prm.N, qx = rc - qy * prm.N;
    const int h = w / 2, n = w * w;
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
    for (int cy = max(qy - h, 0); cy <= min(qy + h, prm.M - 1); ++cy) {
        for (int cx = max(qx - h, 0); cx <= min(qx + h, prm.N - 1); ++cx) {
            const size_t cpix = ((size_t)b * prm.M + cy) * prm.N + cx;
            for (int u = 0; u < n; ++u) {
                const int sy = min(max(cy + u / w - h, 0), prm.M - 1);
                const int sx = min(max(cx + u % w - h, 0), prm.N - 1);
                if (sy != qy || sx != qx) continue;
                const float* g = prm.ws + (cpix * n + u) * 3;
                a0 += g[0];
                a1 += g[1];
                a2 += g[2];
            }
        }
    }
    prm.dx[pix * 3 + 0] = a0;
    prm.dx[pix * 3 + 1] = a1;
    prm.dx[pix * 3 + 2] = a2;
}

template <int KIND>
static hipError_t launch_soft_direct(int w, bool bwd, const SoftParams& prm, hipStream_t s) {
    SoftParams q = prm;
    const long long npix = (long long)prm.B * prm.M * prm.N;
    const long long nblk = (npix + kSoftDirThreads - 1) / kSoftDirThreads;
    q.grid = tile_grid(1, (int)nblk, 1);
    const dim3 grid = flat_grid(nblk), block(kSoftDirThreads);
    if (!bwd) {
        hipLaunchKernelGGL((softmin_direct_kernel<KIND, false>), grid, block, 0, s, q, w);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((softmin_direct_kernel<KIND, true>), grid, block, 0, s, q, w);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(softmin_direct_gather, grid, block, 0, s, q, w);
    return hipGetLastError();
}

template <int W, int KIND, bool BWD>
static void soft_grid(const SoftParams& prm, int& tx, int& ty, int& nt) {
    using Gm = FwdGeom<W, SoftTile<W, KIND, BWD>::EXT_W, SoftTile<W, KIND, BWD>::EXT_H>;
    tx = (prm.N + Gm::TW - 1) / Gm::TW;
    ty = (prm.M + Gm::TH - 1) / Gm::TH;
    nt = Gm::NT;
}

template <int W, int KIND>
static hipError_t launch_soft_t(bool bwd, const SoftParams& prm, hipStream_t s) {
    int nt;
    SoftParams q = prm;
    if (!bwd) {
        soft_grid<W, KIND, false>(prm, q.tiles_x, q.tiles_y, nt);
        q.grid = tile_grid(prm.B, q.tiles_x, q.tiles_y);
        hipLaunchKernelGGL((softmin_kernel<W, KIND, false>), flat_grid(q.grid.n), dim3(nt), 0, s,
                           q);
        return hipGetLastError();
    }
    soft_grid<W, KIND, true>(prm, q.tiles_x, q.tiles_y, nt);
    q.grid = tile_grid(prm.B, q.tiles_x, q.tiles_y);
    q.cgrid = tile_grid(prm.B, (prm.N + 63) / 64, (prm.M + 3) / 4);
    hipLaunchKernelGGL((softmin_kernel<W, KIND, true>), flat_grid(q.grid.n), dim3(nt), 0, s, q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((softmin_combine<W, KIND>), flat_grid(q.cgrid.n), dim3(256), 0, s, q);
    return hipGetLastError();
}

size_t softmin_workspace_bytes(int window, int kind, int B, int M, int N) {
    if (window >= 11)  // the direct form: n x 3 floats per pixel
        return (size_t)B * M * N * window * window * 3 * sizeof(float);
    SoftParams prm{};
    prm.B = B; prm.M = M; prm.N = N;
    int tx, ty, nt;
    if (window == 3) {
        if (kind == kBVDF) soft_grid<3, kBVDF, true>(prm, tx, ty, nt);
        else soft_grid<3, kDDF, true>(prm, tx, ty, nt);
    } else if (window == 5) {
        if (kind == kBVDF) soft_grid<5, kBVDF, true>(prm, tx, ty, nt);
        else soft_grid<5, kDDF, true>(prm, tx, ty, nt);
    } else if (window == 7) {
        if (kind == kBVDF) soft_grid<7, kBVDF, true>(prm, tx, ty, nt);
        else soft_grid<7, kDDF, true>(prm, tx, ty, nt);
    } else {
        if (kind == kBVDF) soft_grid<9, kBVDF, true>(prm, tx, ty, nt);
        else soft_grid<9, kDDF, true>(prm, tx, ty, nt);
    }
    return (size_t)B * tx * ty * nt * 3 * sizeof(float);
}

hipError_t launch_softmin(int window, int kind, bool bwd, const SoftParams& prm, hipStream_t s) {
    if (window >= 11)
        return kind == kBVDF ? launch_soft_direct<kBVDF>(window, bwd, prm, s)
                             : launch_soft_direct<kDDF>(window, bwd, prm, s);
    if (window == 3)
        return kind == kBVDF ? launch_soft_t<3, kBVDF>(bwd, prm, s) : launch_soft_t<3, kDDF>(bwd, prm, s);
    if (window == 5)
        return kind == kBVDF ? launch_soft_t<5, kBVDF>(bwd, prm, s) : launch_soft_t<5, kDDF>(bwd, prm, s);
    if (window == 7)
        return kind == kBVDF ? launch_soft_t<7, kBVDF>(bwd, prm, s) : launch_soft_t<7, kDDF>(bwd, prm, s);
    return kind == kBVDF ? launch_soft_t<9, kBVDF>(bwd, prm, s) : launch_soft_t<9, kDDF>(bwd, prm, s);
}

}  // namespace odf
