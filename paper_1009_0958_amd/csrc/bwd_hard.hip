// bwd_hard.hip -- gradient of the hard (argmin) filter.
//
// The forward output y(c) is a copy of the selected member
// x(clamp(c + offset(u*(c)))), so dL/dx(q) is the sum of dL/dy(c) over the
// windows c whose selection is the pixel q.  Every such c lies within h of q
// (a clamped member stays within h of its window centre), so each thread
// gathers over the (2h+1)^2 windows around its pixel, visiting them in raster
// order and accumulating in binary64: the result is the binary64 raster-order
// sum rounded once to binary32, independent of the launch shape.
#include "odf_internal.h"

namespace odf {

template <int W>
__global__ void __launch_bounds__(256) bwd_hard_kernel(const uint8_t* __restrict__ idx,
                                                       const float* __restrict__ dy,
                                                       float* __restrict__ dx, int M, int N) {
    constexpr int H = W / 2;
    const int gx = blockIdx.x * 64 + (threadIdx.x & 63);
    const int gy = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int b = blockIdx.z;
    if (gx >= N || gy >= M) return;
    const size_t base = (size_t)b * M * N;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const int y0 = max(gy - H, 0), y1 = min(gy + H, M - 1);
    const int x0 = max(gx - H, 0), x1 = min(gx + H, N - 1);
    for (int cy = y0; cy <= y1; ++cy) {
        for (int cx = x0; cx <= x1; ++cx) {
            const size_t c = base + (size_t)cy * N + cx;
            const int u = idx[c];
            const int sy = min(max(cy + u / W - H, 0), M - 1);
            const int sx = min(max(cx + u % W - H, 0), N - 1);
            if (sy == gy && sx == gx) {
                a0 += (double)dy[c * 3 + 0];
                a1 += (double)dy[c * 3 + 1];
                a2 += (double)dy[c * 3 + 2];
            }
        }
    }
    float* o = dx + (base + (size_t)gy * N + gx) * 3;
    o[0] = (float)a0;
    o[1] = (float)a1;
    o[2] = (float)a2;
}

hipError_t launch_backward_hard(int window, const uint8_t* idx, const float* dy, float* dx, int B,
                                int M, int N, hipStream_t stream) {
    dim3 grid((N + 63) / 64, (M + 3) / 4, B);
    if (window == 3)
        hipLaunchKernelGGL(bwd_hard_kernel<3>, grid, dim3(256), 0, stream, idx, dy, dx, M, N);
    else if (window == 5)
        hipLaunchKernelGGL(bwd_hard_kernel<5>, grid, dim3(256), 0, stream, idx, dy, dx, M, N);
    else
        hipLaunchKernelGGL(bwd_hard_kernel<7>, grid, dim3(256), 0, stream, idx, dy, dx, M, N);
    return hipGetLastError();
}

}  // namespace odf
