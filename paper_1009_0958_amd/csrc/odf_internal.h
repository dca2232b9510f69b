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
};

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
};

hipError_t launch_backward_hard(int window, const uint8_t* idx, const float* dy, float* dx, int B,
                                int M, int N, hipStream_t stream);
size_t softmin_workspace_bytes(int window, int kind, int B, int M, int N);
hipError_t launch_softmin(int window, int kind, bool bwd, const SoftParams& prm, hipStream_t s);

}  // namespace odf
