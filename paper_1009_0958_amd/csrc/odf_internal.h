// odf_internal.h -- launch parameters shared by the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pair_terms.h"

namespace odf {

struct FwdParams {
    const void* img;      // B x M x N x 3, uint8 or float32
    void* out;            // same type and shape as img (may be null in aggregate mode)
    uint8_t* idx;         // B x M x N or null
    float* dbg_A;         // aggregate mode: B x M x N x n (null otherwise)
    float* dbg_D;
    float* dbg_O;
    int B, M, N;
    float p;              // DDF weight
    MinimaxCoef coef;     // Table 1 row for the chosen q
    // ACWDDF: extra weight of the centre term, w_d(k) - 1 = n - 2k + 1, at the
    // levels k = lambda, lambda + 1, lambda + 2, and the switching threshold T
    float acw_wm1[3];
    float acw_T;
    int tiles_x, tiles_y;  // output tiles across and down one image (set by the launch)
};

// Workgroup grids.  A launch of n workgroups (1 <= n < 2^31) takes x = min(n, 65535)
// and y = ceil(n / x) < 32768: inside the dispatch limits on every dimension and on
// work-items per dimension, however the images are shaped (2^31 one-pixel images,
// one 2^31-pixel row).  The hardware dispatches x fastest, so flat_block(n) numbers
// the workgroups in dispatch order; it is -1 for those at or past n (the tail of the
// last row), which have no work and return at once.
constexpr int kGridX = 65535;
inline dim3 flat_grid(long long n) {
    const long long gx = n < 1 ? 1 : (n < kGridX ? n : kGridX);
    return dim3((unsigned)gx, (unsigned)((n + gx - 1) / gx));
}
__device__ __forceinline__ int flat_block(int n) {
    // below 2^31 + 65535: no unsigned wrap, and compared before it is made an int
    const unsigned t = blockIdx.y * gridDim.x + blockIdx.x;
    return t < (unsigned)n ? (int)t : -1;
}

// Tile t of B images of tiles_x x tiles_y tiles each, numbered image by image and
// row by row within an image (the order of a (tiles_x, tiles_y, B) grid).
struct TileCoord {
    int b, ty, tx;
};
__device__ __forceinline__ TileCoord tile_coord(int t, int tiles_x, int tiles_y) {
    const int per = tiles_x * tiles_y;
    const int b = t / per, r = t - b * per;
    const int ty = r / tiles_x;
    return {b, ty, r - ty * tiles_x};
}

// Launch the forward filter on `stream` with extended-tile shape `cfg`.
// Returns hipSuccess or the launch error.
hipError_t launch_forward(int window, int kind, int dist, bool u8, bool aggregates, int cfg,
                          const FwdParams& prm, hipStream_t stream);
bool tile_config_valid(int window, int kind, int cfg);
int tile_config_default(int window, int kind);
void tile_config_shape(int cfg, int* ext_w, int* ext_h);
constexpr int kNumTileShapes = 4;
int tuned_config(int window, int kind, int dist, bool u8);
void set_tuned_config(int window, int kind, int dist, bool u8, int cfg);

// Table 1 coefficients for degree q (zeros outside 2..4).
MinimaxCoef minimax_coef(int q);

// ACWDDF fields of prm for window w, level lambda and threshold T.
void set_acw_params(int window, int lambda, float T, FwdParams& prm);

// Record the message returned by odf_last_error() on this thread; returns code.
int set_error(int code, const char* fmt, ...);

struct SoftParams {
    const float* x;   // B x M x N x 3
    const float* dy;  // backward: upstream gradient, B x M x N x 3
    float* y;         // forward output
    float* dx;        // backward output
    float* ws;        // backward workspace (per-tile contributions)
    int B, M, N;
    float p;
    float inv_tau;
    int tiles_x, tiles_y;  // tiles across and down one image (set by the launch)
};

hipError_t launch_backward_hard(int window, const uint8_t* idx, const float* dy, float* dx, int B,
                                int M, int N, hipStream_t stream);
size_t softmin_workspace_bytes(int window, int kind, int B, int M, int N);
hipError_t launch_softmin(int window, int kind, bool bwd, const SoftParams& prm, hipStream_t s);

}  // namespace odf
