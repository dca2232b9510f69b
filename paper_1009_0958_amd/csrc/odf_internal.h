// odf_internal.h -- launch parameters shared by the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pair_terms.h"

namespace odf {

// Workgroup grids.  A launch of n workgroups (1 <= n < 2^31) takes y = ceil(n / 65535)
// rows (<= 32769) of x = ceil(n / y) <= 65535 workgroups: inside the dispatch limits on
// every dimension and on work-items per dimension, however the images are shaped
// (2^31 one-pixel images, one 2^31-pixel row), and fewer than y workgroups past n
// (x = 65535 for n just above 65535 would launch up to 65534 idle ones, measured at
// 5 % of a 3x3 launch).  The hardware dispatches x fastest, so flat_block(n) numbers
// the workgroups in dispatch order; it is -1 for those at or past n, which have no
// work and return at once.
constexpr int kGridX = 65535;
inline dim3 flat_grid(long long n) {
    if (n < 1) n = 1;
    const long long gy = (n + kGridX - 1) / kGridX;
    return dim3((unsigned)((n + gy - 1) / gy), (unsigned)gy);
}
__device__ __forceinline__ int flat_block(int n) {
    // below 2^31 + 32769: no unsigned wrap, and compared before it is made an int
    const unsigned t = blockIdx.y * gridDim.x + blockIdx.x;
    return t < (unsigned)n ? (int)t : -1;
}

// XCD-contiguous numbering of a launch's n workgroups: the hardware hands the
// workgroup of dispatch index t0 to XCD t0 mod 8 (each with its own L2), so
// item xcd_item(t0, n) = (first item of that XCD) + t0 / 8 gives every XCD one
// contiguous run of items (a bijection of [0, n)): neighbouring items then
// share their halo and the cache lines they straddle in one L2.
__device__ __forceinline__ int xcd_item(int t0, int n) {
    const int q = n / 8, r = n - 8 * q, x = t0 % 8;
    return x * q + min(x, r) + t0 / 8;
}

// Division of a 32-bit unsigned integer by a divisor fixed for a launch, as a
// multiply-high, a subtraction, an addition and two shifts on uniform values
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994, Figure 4.1): with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, t = mulhi(m, n) gives
// n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0) for every 32-bit n.
// The compiler's own division by a runtime value costs ~20 vector
// instructions per wave, a measurable share of a small kernel.
struct FastDiv {
    uint32_t d, m, s1, s2;
};
inline FastDiv fast_div(uint32_t d) {  // d >= 1
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    const uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
    return {d, (uint32_t)m, l < 1 ? l : 1u, l > 1 ? l - 1 : 0u};
}
__device__ __forceinline__ uint32_t div_fast(uint32_t n, const FastDiv& f) {
    const uint32_t t = __umulhi(f.m, n);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

// The tiles of B images of tiles_x x tiles_y tiles each, numbered image by
// image and row by row within an image (the order of a (tiles_x, tiles_y, B)
// grid); n = B tiles_x tiles_y < 2^31.
struct TileGrid {
    int n;
    FastDiv per_image, across;
};
inline TileGrid tile_grid(int B, int tiles_x, int tiles_y) {
    return {B * tiles_x * tiles_y, fast_div((uint32_t)(tiles_x * tiles_y)),
            fast_div((uint32_t)tiles_x)};
}
struct TileCoord {
    int b, ty, tx;
};
__device__ __forceinline__ TileCoord tile_coord(int t, const TileGrid& g) {
    const uint32_t b = div_fast((uint32_t)t, g.per_image);
    const uint32_t r = (uint32_t)t - b * g.per_image.d;
    const uint32_t ty = div_fast(r, g.across);
    return {(int)b, (int)ty, (int)(r - ty * g.across.d)};
}

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
    TileGrid grid;    // the launch's tiles (set by the launch)
    int strip_bands;  // strip form: bands per strip (set by the launch)
};

// Launch the forward filter on `stream` with extended-tile shape `cfg`.
// Returns hipSuccess or the launch error.
hipError_t launch_forward(int window, int kind, int dist, bool u8, bool aggregates, int cfg,
                          const FwdParams& prm, hipStream_t stream);
bool tile_config_valid(int window, int kind, int cfg, bool u8);
int tile_config_default(int window, int kind);
void tile_config_shape(int cfg, int* ext_w, int* ext_h);
constexpr int kNumTileShapes = 4;
// Forward configs: the four tile shapes, then the strip form (fwd_strip.h:
// 32-wide strips of bands of 16 rows): 8 bands per strip, or 3 for images too
// small to fill the GPU with the long strips.
constexpr int kStripConfig = 4;
constexpr int kShortStripConfig = 5;
constexpr int kNumTileConfigs = 6;
constexpr bool is_strip_config(int cfg) { return cfg == kStripConfig || cfg == kShortStripConfig; }
constexpr int strip_bands(int cfg) { return cfg == kShortStripConfig ? 3 : 8; }
// Extended-tile shapes (EXT_W x EXT_H, one thread per extended pixel) the
// autotuners choose from, for the per-image and the batch kernels alike.
constexpr int kTileW[kNumTileShapes] = {32, 64, 32, 64};
constexpr int kTileH[kNumTileShapes] = {32, 16, 16, 8};
// The batch kernels' shape per group (window 3 / 5 x BVDF / DDF, group =
// (window == 5) * 2 + kind): the process-wide batch tuning table.
// Batch groups: one per (window 3, 5, 7 or 9, kind BVDF or DDF), numbered
// ((window - 3) / 2) * 2 + kind; classes add the pair term: group * 3 + dist.
constexpr int kNumBatchGroups = 8;
inline bool batch_window(int window) {
    return window == 3 || window == 5 || window == 7 || window == 9;
}
inline int batch_group(int window, int kind) { return (window - 3) / 2 * 2 + (kind == kDDF); }
inline int batch_group_window(int group) { return 3 + 2 * (group / 2); }
int batch_tuned_config(int group);
void set_batch_tuned_config(int group, int cfg);
// A seeded uint8 tuning image (M x N x 3): a smooth field of a few plane
// waves per channel with 15 % of the pixels replaced by random colours, the
// kind of content the filters meet (their branches -- the minimax z = 1/2
// test, the zero-pixel fix-ups -- depend on it).
void tuning_image(int M, int N, uint64_t seed, uint8_t* out);
// Tile table entry of (window, kind, dist, input type), kind the C ABI's
// odf_kind; kernel_kind maps an odf_kind to the kernels' Kind.
int tuned_config(int window, int kind, int dist, bool u8);
void set_tuned_config(int window, int kind, int dist, bool u8, int cfg);
int kernel_kind(int kind);

// Table 1 coefficients for degree q (zeros outside 2..4).
MinimaxCoef minimax_coef(int q);

// ACWDDF fields of prm for window w, level lambda and threshold T.
void set_acw_params(int window, int lambda, float T, FwdParams& prm);

// Record the message returned by odf_last_error() on this thread; returns code.
int set_error(int code, const char* fmt, ...);

// Allocation-failure injection for tests: true when the environment variable
// ODF_TEST_FAIL_ALLOC is set to anything but "" or "0".  The calls that
// allocate (odf_batch_plan, odf_autotune) then take their allocation-failure
// path (ODF_ENOMEM) before allocating or touching the device.
bool test_fail_alloc();

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
    TileGrid grid;         // the launch's tiles (set by the launch)
    TileGrid cgrid;        // the combine pass's 64 x 4 pixel blocks
};

// BVDF / DDF at the odd windows 11 to 15 (general.hip: a direct form, no tile
// configs), and the hard backward at any odd window up to 15.
hipError_t launch_forward_general(int window, int kind, int dist, bool u8, const FwdParams& prm,
                                  hipStream_t stream);
hipError_t launch_backward_hard_general(int window, const uint8_t* idx, const float* dy, float* dx,
                                        int B, int M, int N, hipStream_t stream);
hipError_t launch_backward_hard(int window, const uint8_t* idx, const float* dy, float* dx, int B,
                                int M, int N, hipStream_t stream);
size_t softmin_workspace_bytes(int window, int kind, int B, int M, int N);
hipError_t launch_softmin(int window, int kind, bool bwd, const SoftParams& prm, hipStream_t s);

}  // namespace odf
