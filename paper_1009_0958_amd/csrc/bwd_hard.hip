// bwd_hard.hip -- gradient of the hard (argmin) filter.
//
// The forward output y(c) is a copy of the selected member
// x(clamp(c + offset(u*(c)))), so dL/dx(q) is the sum of dL/dy(c) over the
// windows c whose selection is the pixel q.  Every such c lies within h of q
// (a clamped member stays within h of its window centre).  A workgroup owns a
// 64 x 8 tile of q (two rows per thread): it stages, for the tile and its
// h-halo, each window's selected pixel (as a local index, computed once per
// window) and dy(c) in LDS; each thread then visits the (2h+1)^2 windows around its pixel in raster
// order and accumulates in binary64, so the result is the binary64
// raster-order sum rounded once to binary32, independent of the launch shape.
#include "odf_internal.h"

namespace odf {

// 64 x 8 re-reads less halo than 64 x 4 (1.6 instead of 2.1 staged cells per
// pixel at 5x5) and measured 2-6 % faster; 64 x 16 (four rows per thread)
// measured slower: fewer workgroups to hide the latency of the staging loads
constexpr int kBwdTW = 64, kBwdTH = 8, kBwdRowsPerThread = kBwdTH / 4;

template <int W>
__global__ void __launch_bounds__(256) bwd_hard_kernel(const uint8_t* __restrict__ idx,
                                                       const float* __restrict__ dy,
                                                       float* __restrict__ dx, int M, int N,
                                                       TileGrid grid) {
    constexpr int H = W / 2, RW = kBwdTW + 2 * H, RH = kBwdTH + 2 * H, RN = RW * RH;
    __shared__ int s_tgt[RN];       // local index of the pixel window c selects, or -1
    __shared__ float s_dy[3 * RN];  // dy(c)
    const int tile = flat_block(grid.n);
    if (tile < 0) return;
    const TileCoord tc = tile_coord(tile, grid);
    const int tx0 = tc.tx * kBwdTW, ty0 = tc.ty * kBwdTH;
    const size_t base = (size_t)tc.b * M * N;
    for (int i = threadIdx.x; i < RN; i += blockDim.x) {
        const int ry = i / RW, rx = i - ry * RW;
        const int cy = ty0 - H + ry, cx = tx0 - H + rx;
        int t = -1;
        float d0 = 0.0f, d1 = 0.0f, d2 = 0.0f;
        if (cy >= 0 && cy < M && cx >= 0 && cx < N) {
            const size_t c = base + (size_t)cy * N + cx;
            const int u = idx[c];
            const int sy = min(max(cy + u / W - H, 0), M - 1) - (ty0 - H);
            const int sx = min(max(cx + u % W - H, 0), N - 1) - (tx0 - H);
            if (sy >= 0 && sy < RH && sx >= 0 && sx < RW) t = sy * RW + sx;
            d0 = dy[c * 3 + 0];
            d1 = dy[c * 3 + 1];
            d2 = dy[c * 3 + 2];
        }
        s_tgt[i] = t;
        s_dy[3 * i + 0] = d0;
        s_dy[3 * i + 1] = d1;
        s_dy[3 * i + 2] = d2;
    }
    __syncthreads();
    const int lx = threadIdx.x % kBwdTW;
    const int gx = tx0 + lx;
    if (gx >= N) return;
    for (int k = 0; k < kBwdRowsPerThread; ++k) {
        const int ly = threadIdx.x / kBwdTW + 4 * k;
        const int gy = ty0 + ly;
        if (gy >= M) break;
        const int me = (ly + H) * RW + lx + H;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int oy = -H; oy <= H; ++oy) {
#pragma unroll
            for (int ox = -H; ox <= H; ++ox) {
                const int cell = me + oy * RW + ox;
                if (s_tgt[cell] == me) {
                    a0 += (double)s_dy[3 * cell + 0];
                    a1 += (double)s_dy[3 * cell + 1];
                    a2 += (double)s_dy[3 * cell + 2];
                }
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
    if (window == 3)
        hipLaunchKernelGGL(bwd_hard_kernel<3>, grid, dim3(256), 0, stream, idx, dy, dx, M, N, tg);
    else if (window == 5)
        hipLaunchKernelGGL(bwd_hard_kernel<5>, grid, dim3(256), 0, stream, idx, dy, dx, M, N, tg);
    else
        hipLaunchKernelGGL(bwd_hard_kernel<7>, grid, dim3(256), 0, stream, idx, dy, dx, M, N, tg);
    return hipGetLastError();
}

}  // namespace odf
