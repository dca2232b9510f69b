// bwd_hard.hip -- gradient of the hard (argmin) filter.
//
// The forward output y(c) is a copy of the selected member
// x(clamp(c + offset(u*(c)))), so dL/dx(q) is the sum of dL/dy(c) over the
// windows c whose selection is the pixel q.  Every such c lies within h of q
// (a clamped member stays within h of its window centre).
//
// A workgroup owns a 64 x 8 tile of q (two rows per thread).  It reads, for the
// tile and its h-halo, the index map (one byte per window) and dy into LDS.  Each
// window c whose selection t falls inside the tile sets bit (c - t + (h, h)) of
// t's (2h+1)^2-bit mask with an LDS atomic OR; the bit order is the raster
// order of c.  Each pixel then visits only the windows its mask names, lowest
// bit first, and accumulates their dy in binary64: the binary64 raster-order
// sum rounded once to binary32, independent of the launch shape and of the
// order of the atomics.
#include "odf_internal.h"

namespace odf {

// 64 x 8 re-reads less halo than 64 x 4 (1.6 instead of 2.1 staged cells per
// pixel at 5x5); 64 x 16 (four rows per thread) measured slower: fewer
// workgroups to hide the latency of the staging loads
constexpr int kBwdTW = 64, kBwdTH = 8, kBwdThreads = 256;

template <int W>
__global__ void __launch_bounds__(kBwdThreads) bwd_hard_kernel(const uint8_t* __restrict__ idx,
                                                               const float* __restrict__ dy,
                                                               float* __restrict__ dx, int M,
                                                               int N, TileGrid grid) {
    constexpr int H = W / 2, RW = kBwdTW + 2 * H, RH = kBwdTH + 2 * H, RN = RW * RH;
    constexpr int NB = W * W, WORDS = (NB + 31) / 32;  // mask bits per pixel, 32-bit words
    constexpr int TP = kBwdTW * kBwdTH;                // pixels of the tile
    __shared__ uint32_t s_mask[WORDS * TP];            // word k of pixel l at k * TP + l
    __shared__ float s_dy[3 * RN];                     // dy(c), 3 floats per staged window
    const int t0 = flat_block(grid.n);
    if (t0 < 0) return;
    // XCD-contiguous order: the halo a tile shares with its neighbours is read
    // once per XCD's L2 (HBM traffic 1.24 -> 1.00 times the 25 B per pixel)
    const TileCoord tc = tile_coord(xcd_item(t0, grid.n), grid);
    const int tx0 = tc.tx * kBwdTW, ty0 = tc.ty * kBwdTH;
    const size_t base = (size_t)tc.b * M * N;
    const int tid = threadIdx.x;

    for (int i = tid; i < WORDS * TP; i += kBwdThreads) s_mask[i] = 0u;
    // Every global load of the staging is issued before the first one is used:
    // per staged window its index byte and its dy (three consecutive floats, so
    // a wave reads one contiguous run per row of the region).
    constexpr int NI = (RN + kBwdThreads - 1) / kBwdThreads;
    int u[NI];
    float d[NI][3];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int i = tid + k * kBwdThreads;
        const int ry = i / RW, rx = i - ry * RW;
        const int cy = ty0 - H + ry, cx = tx0 - H + rx;
        u[k] = NB;  // no window: routes nothing
        d[k][0] = d[k][1] = d[k][2] = 0.0f;
        if (i < RN && cy >= 0 && cy < M && cx >= 0 && cx < N) {
            const size_t c = base + (size_t)cy * N + cx;
            u[k] = idx[c];
            d[k][0] = dy[3 * c + 0];
            d[k][1] = dy[3 * c + 1];
            d[k][2] = dy[3 * c + 2];
        }
    }
    __syncthreads();  // masks cleared
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int i = tid + k * kBwdThreads;
        if (i < RN) {
            s_dy[3 * i + 0] = d[k][0];
            s_dy[3 * i + 1] = d[k][1];
            s_dy[3 * i + 2] = d[k][2];
        }
        if (u[k] >= NB) continue;  // outside the image, or not an index of this window size
        const int ry = i / RW, rx = i - ry * RW;
        const int cy = ty0 - H + ry, cx = tx0 - H + rx;
        const int sy = min(max(cy + u[k] / W - H, 0), M - 1);
        const int sx = min(max(cx + u[k] % W - H, 0), N - 1);
        const int ly = sy - ty0, lx = sx - tx0;
        if (ly < 0 || ly >= kBwdTH || lx < 0 || lx >= kBwdTW) continue;  // another tile's pixel
        // c - t lies in [-h, h]^2: the clamped selection stays within h of c
        const int bit = (cy - sy + H) * W + (cx - sx + H);
        atomicOr(&s_mask[(bit >> 5) * TP + ly * kBwdTW + lx], 1u << (bit & 31));
    }
    __syncthreads();
    const int lx = tid % kBwdTW, gx = tx0 + lx;
    if (gx >= N) return;
#pragma unroll
    for (int r = 0; r < kBwdTH / (kBwdThreads / kBwdTW); ++r) {
        const int ly = tid / kBwdTW + r * (kBwdThreads / kBwdTW), gy = ty0 + ly;
        if (gy >= M) break;
        const int l = ly * kBwdTW + lx;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int k = 0; k < WORDS; ++k) {
            uint32_t m = s_mask[k * TP + l];
            while (m) {
                const int bit = 32 * k + __builtin_ctz(m);
                m &= m - 1u;
                const int oy = bit / W - H, ox = bit % W - H;  // c = q + (oy, ox)
                const int cell = (ly + H + oy) * RW + (lx + H + ox);
                a0 += (double)s_dy[3 * cell + 0];
                a1 += (double)s_dy[3 * cell + 1];
                a2 += (double)s_dy[3 * cell + 2];
            }
        }
        float* o = dx + (base + (size_t)gy * N + gx) * 3;
        o[0] = (float)a0;
        o[1] = (float)a1;
        o[2] = (float)a2;
    }
}

hipError_t launch_backward_hard(int window, const uint8_t* idx, const float* dy, float* dx, int B,
                                int M, int N, hipStream_t stream) {
    const TileGrid tg = tile_grid(B, (N + kBwdTW - 1) / kBwdTW, (M + kBwdTH - 1) / kBwdTH);
    const dim3 grid = flat_grid(tg.n);
    const dim3 block(kBwdThreads);
    if (window == 3)
        hipLaunchKernelGGL(bwd_hard_kernel<3>, grid, block, 0, stream, idx, dy, dx, M, N, tg);
    else if (window == 5)
        hipLaunchKernelGGL(bwd_hard_kernel<5>, grid, block, 0, stream, idx, dy, dx, M, N, tg);
    else if (window == 7)
        hipLaunchKernelGGL(bwd_hard_kernel<7>, grid, block, 0, stream, idx, dy, dx, M, N, tg);
    else if (window == 9)
        hipLaunchKernelGGL(bwd_hard_kernel<9>, grid, block, 0, stream, idx, dy, dx, M, N, tg);
    else
        return launch_backward_hard_general(window, idx, dy, dx, B, M, N, stream);
    return hipGetLastError();
}

}  // namespace odf
