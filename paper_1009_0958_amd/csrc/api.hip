// api.hip -- host side of libodf: argument validation, error reporting and
// dispatch to the kernels.  Declarations and contracts: include/odf.h.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "odf.h"
#include "odf_internal.h"

namespace {
thread_local char g_err[512] = "";
}  // namespace

namespace odf {
int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}
bool test_fail_alloc() {
    const char* v = getenv("ODF_TEST_FAIL_ALLOC");
    return v && *v && strcmp(v, "0") != 0;
}
}  // namespace odf

namespace {

using odf::set_error;
#define fail set_error

int hip_fail(hipError_t e, const char* what) {
    return fail(ODF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    if (!a || !b || na == 0 || nb == 0) return false;
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

// Table 1 (Section 2.1): minimax coefficients a_0..a_4, rows q = 2, 3, 4.
const float kTab1Asin[3][5] = {
    {1.829125e-03f, 1.371117f, 1.480266e-01f, 0.0f, 0.0f},
    {-1.358425e-04f, 1.419488f, -3.090315e-02f, 1.666491e-01f, 0.0f},
    {2.097797e-05f, 1.412840f, 1.429881e-02f, 6.704361e-02f, 6.909677e-02f},
};
const float kTab1Acos[3][5] = {
    {1.569882f, -9.695260e-01f, -1.480266e-01f, 0.0f, 0.0f},
    {1.570864f, -1.003730f, 3.090318e-02f, -2.356775e-01f, 0.0f},
    {1.570786f, -9.990285e-01f, -1.429899e-02f, -9.481335e-02f, -1.381942e-01f},
};

int check_common(const void* img, int B, int M, int N, int window, int kind, float p, int dist,
                 int q) {
    if (!img) return fail(ODF_EINVAL, "img is NULL");
    if (B < 1 || M < 1 || N < 1) return fail(ODF_EINVAL, "sizes must be >= 1 (B=%d M=%d N=%d)", B, M, N);
    if ((long long)B * M * N >= (1ll << 31))
        return fail(ODF_EINVAL, "B*M*N must be < 2^31 pixels");
    if (window < 3 || window > 15 || window % 2 == 0)
        return fail(ODF_EUNSUPPORTED, "window %d not supported (odd, 3 to 15)", window);
    if (kind != ODF_BVDF && kind != ODF_DDF) return fail(ODF_EINVAL, "kind %d out of range", kind);
    if (dist < ODF_EXACT || dist > ODF_RGB) return fail(ODF_EINVAL, "dist %d out of range", dist);
    if (dist == ODF_MINIMAX && (q < 2 || q > 4))
        return fail(ODF_EINVAL, "q %d out of range (2, 3 or 4)", q);
    if (kind == ODF_DDF && !(p >= 0.0f && p <= 1.0f))
        return fail(ODF_EINVAL, "p must lie in [0, 1] for DDF");
    return ODF_OK;
}

}  // namespace

odf::MinimaxCoef odf::minimax_coef(int q) {
    MinimaxCoef c{};
    if (q >= 2 && q <= 4) {
        memcpy(c.asin_c, kTab1Asin[q - 2], sizeof c.asin_c);
        memcpy(c.acos_c, kTab1Acos[q - 2], sizeof c.acos_c);
    }
    return c;
}

void odf::set_acw_params(int window, int lambda, float T, FwdParams& prm) {
    const int n = window * window;
    for (int j = 0; j < 3; ++j) prm.acw_wm1[j] = (float)(n - 2 * (lambda + j) + 1);
    prm.acw_T = T;
}

namespace {

odf::FwdParams make_params(const void* img, int B, int M, int N, float p, int dist, int q) {
    odf::FwdParams prm{};
    prm.img = img;
    prm.B = B;
    prm.M = M;
    prm.N = N;
    prm.p = p;
    if (dist == ODF_MINIMAX) prm.coef = odf::minimax_coef(q);
    return prm;
}

int filter_any(const void* img, bool u8, int B, int M, int N, int window, int kind, float p,
               int dist, int q, void* out, uint8_t* idx, void* stream) {
    int rc = check_common(img, B, M, N, window, kind, p, dist, q);
    if (rc) return rc;
    if (!out) return fail(ODF_EINVAL, "out is NULL");
    const size_t npix = (size_t)B * M * N;
    const size_t esz = u8 ? 1 : 4;
    if (overlaps(img, npix * 3 * esz, out, npix * 3 * esz))
        return fail(ODF_EINVAL, "out overlaps img (the filter cannot run in place)");
    if (idx && (overlaps(img, npix * 3 * esz, idx, npix) || overlaps(out, npix * 3 * esz, idx, npix)))
        return fail(ODF_EINVAL, "idx overlaps img or out");
    odf::FwdParams prm = make_params(img, B, M, N, kind == ODF_DDF ? p : 0.0f, dist, q);
    prm.out = out;
    prm.idx = idx;
    // windows past 9x9 run the direct form, which has no tile configs
    const int cfg = window <= 9 ? odf::tuned_config(window, kind, dist, u8) : 0;
    hipError_t e = odf::launch_forward(window, kind, dist, u8, false, cfg, prm,
                                       static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return ODF_OK;
}

int acwddf_any(const void* img, bool u8, int B, int M, int N, int window, int dist, int q,
               int lambda, float T, void* out, uint8_t* idx, void* stream) {
    int rc = check_common(img, B, M, N, window, ODF_DDF, 0.5f, dist, q);
    if (rc) return rc;
    if (!out) return fail(ODF_EINVAL, "out is NULL");
    const int dmax = (window * window + 1) / 2 - 2;
    if (lambda < 1 || lambda > dmax)
        return fail(ODF_EINVAL, "lambda %d out of range [1, %d]", lambda, dmax);
    if (T != T) return fail(ODF_EINVAL, "T is NaN");
    const size_t npix = (size_t)B * M * N;
    const size_t esz = u8 ? 1 : 4;
    if (overlaps(img, npix * 3 * esz, out, npix * 3 * esz))
        return fail(ODF_EINVAL, "out overlaps img (the filter cannot run in place)");
    if (idx && (overlaps(img, npix * 3 * esz, idx, npix) || overlaps(out, npix * 3 * esz, idx, npix)))
        return fail(ODF_EINVAL, "idx overlaps img or out");
    odf::FwdParams prm = make_params(img, B, M, N, 0.5f, dist, q);
    prm.out = out;
    prm.idx = idx;
    odf::set_acw_params(window, lambda, T, prm);
    // from 9x9 the centre-weighted kinds run the direct form, which has no configs
    const int cfg = window <= 7 ? odf::tuned_config(window, ODF_ACWDDF, dist, u8) : 0;
    hipError_t e = odf::launch_forward(window, ODF_ACWDDF, dist, u8, false, cfg, prm,
                                       static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "ACWDDF launch");
    return ODF_OK;
}

int cw_any(const void* img, bool u8, int B, int M, int N, int window, int kind, int dist, int q,
           int level, void* out, uint8_t* idx, void* stream) {
    int rc = check_common(img, B, M, N, window, ODF_DDF, 0.5f, dist, q);
    if (rc) return rc;
    if (kind != ODF_CWVMF && kind != ODF_CWDDF)
        return fail(ODF_EINVAL, "kind %d is not ODF_CWVMF or ODF_CWDDF", kind);
    if (!out) return fail(ODF_EINVAL, "out is NULL");
    const int n = window * window, dmax = (n + 1) / 2;
    if (level < 1 || level > dmax) return fail(ODF_EINVAL, "level %d out of range [1, %d]", level, dmax);
    const size_t npix = (size_t)B * M * N;
    const size_t esz = u8 ? 1 : 4;
    if (overlaps(img, npix * 3 * esz, out, npix * 3 * esz))
        return fail(ODF_EINVAL, "out overlaps img (the filter cannot run in place)");
    if (idx && (overlaps(img, npix * 3 * esz, idx, npix) || overlaps(out, npix * 3 * esz, idx, npix)))
        return fail(ODF_EINVAL, "idx overlaps img or out");
    // CWVMF^k has no angle term: its kernel sweeps the L2 term alone
    const int d = kind == ODF_CWVMF ? ODF_RGB : dist;
    odf::FwdParams prm = make_params(img, B, M, N, 0.5f, d, q);
    prm.out = out;
    prm.idx = idx;
    for (int j = 0; j < 3; ++j) prm.acw_wm1[j] = (float)(n - 2 * level + 1);  // w_d(k) - 1
    const int cfg = window <= 7 ? odf::tuned_config(window, kind, d, u8) : 0;
    hipError_t e = odf::launch_forward(window, odf::kernel_kind(kind), d, u8, false, cfg, prm,
                                       static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "centre-weighted filter launch");
    return ODF_OK;
}

}  // namespace

extern "C" {

int odf_version(void) { return (0 << 16) | 3; }

int odf_cw_filter_u8(const uint8_t* img, int B, int M, int N, int window, int kind, int dist, int q,
                     int level, uint8_t* out, uint8_t* idx, void* stream) {
    return cw_any(img, true, B, M, N, window, kind, dist, q, level, out, idx, stream);
}

int odf_cw_filter_f32(const float* img, int B, int M, int N, int window, int kind, int dist, int q,
                      int level, float* out, uint8_t* idx, void* stream) {
    return cw_any(img, false, B, M, N, window, kind, dist, q, level, out, idx, stream);
}

int odf_acwddf_u8(const uint8_t* img, int B, int M, int N, int window, int dist, int q,
                  int lambda, float T, uint8_t* out, uint8_t* idx, void* stream) {
    return acwddf_any(img, true, B, M, N, window, dist, q, lambda, T, out, idx, stream);
}

int odf_acwddf_f32(const float* img, int B, int M, int N, int window, int dist, int q,
                   int lambda, float T, float* out, uint8_t* idx, void* stream) {
    return acwddf_any(img, false, B, M, N, window, dist, q, lambda, T, out, idx, stream);
}

const char* odf_last_error(void) { return g_err; }

int odf_filter_u8(const uint8_t* img, int B, int M, int N, int window, int kind, float p, int dist,
                  int q, uint8_t* out, uint8_t* idx, void* stream) {
    return filter_any(img, true, B, M, N, window, kind, p, dist, q, out, idx, stream);
}

int odf_filter_f32(const float* img, int B, int M, int N, int window, int kind, float p, int dist,
                   int q, float* out, uint8_t* idx, void* stream) {
    return filter_any(img, false, B, M, N, window, kind, p, dist, q, out, idx, stream);
}

int odf_aggregates_f32(const void* img, int is_u8, int B, int M, int N, int window, int kind,
                       float p, int dist, int q, float* A, float* D, float* Omega, void* stream) {
    int rc = check_common(img, B, M, N, window, kind, p, dist, q);
    if (rc) return rc;
    if (window > 9) return fail(ODF_EUNSUPPORTED, "aggregates are exported for windows 3 to 9");
    if (!A) return fail(ODF_EINVAL, "A is NULL");
    const size_t npix = (size_t)B * M * N;
    const size_t nagg = npix * window * window * sizeof(float);
    const size_t nimg = npix * 3 * (is_u8 ? 1 : 4);
    if (overlaps(img, nimg, A, nagg) || overlaps(img, nimg, D, nagg) ||
        overlaps(img, nimg, Omega, nagg) || overlaps(A, nagg, D, nagg) ||
        overlaps(A, nagg, Omega, nagg) || overlaps(D, nagg, Omega, nagg))
        return fail(ODF_EINVAL, "output arrays overlap each other or img");
    odf::FwdParams prm = make_params(img, B, M, N, kind == ODF_DDF ? p : 0.0f, dist, q);
    prm.dbg_A = A;
    prm.dbg_D = D;
    prm.dbg_O = Omega;
    hipError_t e = odf::launch_forward(window, kind, dist, is_u8 != 0, true, 0, prm,
                                       static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "aggregate launch");
    return ODF_OK;
}

int odf_backward_hard_f32(const uint8_t* idx, const float* dy, int B, int M, int N, int window,
                          float* dx, void* stream) {
    if (!idx || !dy || !dx) return fail(ODF_EINVAL, "idx, dy and dx must be non-NULL");
    if (B < 1 || M < 1 || N < 1) return fail(ODF_EINVAL, "sizes must be >= 1 (B=%d M=%d N=%d)", B, M, N);
    if ((long long)B * M * N >= (1ll << 31)) return fail(ODF_EINVAL, "B*M*N must be < 2^31 pixels");
    if (window < 3 || window > 15 || window % 2 == 0)
        return fail(ODF_EUNSUPPORTED, "window %d not supported (odd, 3 to 15)", window);
    const size_t npix = (size_t)B * M * N;
    if (overlaps(dx, npix * 12, dy, npix * 12) || overlaps(dx, npix * 12, idx, npix))
        return fail(ODF_EINVAL, "dx overlaps dy or idx");
    hipError_t e = odf::launch_backward_hard(window, idx, dy, dx, B, M, N,
                                             static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "hard backward launch");
    return ODF_OK;
}

static int check_soft(const float* x, int B, int M, int N, int window, int kind, float p, float tau) {
    int rc = check_common(x, B, M, N, window, kind, p, ODF_EXACT, 4);
    if (rc) return rc;
    if (!(tau > 0.0f) || !(tau < 3.0e38f)) return fail(ODF_EINVAL, "tau must be positive and finite");
    return ODF_OK;
}

int odf_softmin_fwd_f32(const float* x, int B, int M, int N, int window, int kind, float p,
                        float tau, float* y, void* stream) {
    int rc = check_soft(x, B, M, N, window, kind, p, tau);
    if (rc) return rc;
    if (!y) return fail(ODF_EINVAL, "y is NULL");
    const size_t nb = (size_t)B * M * N * 12;
    if (overlaps(x, nb, y, nb)) return fail(ODF_EINVAL, "y overlaps x");
    odf::SoftParams prm{};
    prm.x = x; prm.y = y; prm.B = B; prm.M = M; prm.N = N;
    prm.p = kind == ODF_DDF ? p : 0.0f;
    prm.inv_tau = 1.0f / tau;
    hipError_t e = odf::launch_softmin(window, kind, false, prm, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "softmin forward launch");
    return ODF_OK;
}

size_t odf_softmin_bwd_workspace(int B, int M, int N, int window, int kind) {
    if (B < 1 || M < 1 || N < 1 || window < 3 || window > 15 || window % 2 == 0 ||
        (kind != ODF_BVDF && kind != ODF_DDF))
        return 0;
    return odf::softmin_workspace_bytes(window, kind, B, M, N);
}

int odf_softmin_bwd_f32(const float* x, const float* dy, int B, int M, int N, int window, int kind,
                        float p, float tau, float* dx, void* workspace, size_t workspace_bytes,
                        void* stream) {
    int rc = check_soft(x, B, M, N, window, kind, p, tau);
    if (rc) return rc;
    if (!dy || !dx || !workspace) return fail(ODF_EINVAL, "dy, dx and workspace must be non-NULL");
    const size_t need = odf::softmin_workspace_bytes(window, kind, B, M, N);
    if (workspace_bytes < need)
        return fail(ODF_EINVAL, "workspace too small (%zu < %zu bytes)", workspace_bytes, need);
    const size_t nb = (size_t)B * M * N * 12;
    if (overlaps(dx, nb, x, nb) || overlaps(dx, nb, dy, nb) || overlaps(workspace, need, x, nb) ||
        overlaps(workspace, need, dy, nb) || overlaps(workspace, need, dx, nb))
        return fail(ODF_EINVAL, "dx / workspace overlap an input or each other");
    odf::SoftParams prm{};
    prm.x = x; prm.dy = dy; prm.dx = dx; prm.ws = static_cast<float*>(workspace);
    prm.B = B; prm.M = M; prm.N = N;
    prm.p = kind == ODF_DDF ? p : 0.0f;
    prm.inv_tau = 1.0f / tau;
    hipError_t e = odf::launch_softmin(window, kind, true, prm, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "softmin backward launch");
    return ODF_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ static scratch
// Workspace of odf_softmin_bwd_f32_noalloc: a device array of the library, one
// copy on every GPU the library is loaded on, held until the process ends.  Host
// code must not pass `scratch` itself to a kernel or a copy (in host code the
// name stands for a host-side shadow, not a device address): it looks up the
// array's address on the current device once with hipGetSymbolAddress and uses
// that pointer.
namespace {
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices];  // per device ordinal, guarded by g_scratch_mu

// Address of `scratch` on the current device (looked up on the first call on
// each device, with that device current).
int scratch_on_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(ODF_EUNSUPPORTED, "device ordinal %d: the static scratch serves devices 0..%d",
                    dev, kMaxScratchDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(ODF_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return ODF_OK;
}
}  // namespace

extern "C" {

int odf_softmin_bwd_f32_noalloc(const float* x, const float* dy, int B, int M, int N, int window,
                                int kind, float p, float tau, float* dx, void* stream) {
    int rc = check_soft(x, B, M, N, window, kind, p, tau);
    if (rc) return rc;
    if (!dy || !dx) return fail(ODF_EINVAL, "dy and dx must be non-NULL");
    const size_t need = odf::softmin_workspace_bytes(window, kind, B, M, N);
    if (need > kScratchBytes)
        return fail(ODF_EINVAL,
                    "this shape needs %zu bytes of workspace, more than the %zu of the static "
                    "scratch (use odf_softmin_bwd_f32 with a workspace)", need, kScratchBytes);
    const size_t nb = (size_t)B * M * N * 12;
    if (overlaps(dx, nb, x, nb) || overlaps(dx, nb, dy, nb))
        return fail(ODF_EINVAL, "dx overlaps x or dy");
    void* ws = nullptr;
    rc = scratch_on_current_device(&ws);
    if (rc) return rc;
    odf::SoftParams prm{};
    prm.x = x; prm.dy = dy; prm.dx = dx; prm.ws = static_cast<float*>(ws);
    prm.B = B; prm.M = M; prm.N = N;
    prm.p = kind == ODF_DDF ? p : 0.0f;
    prm.inv_tau = 1.0f / tau;
    hipError_t e = odf::launch_softmin(window, kind, true, prm, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "softmin backward launch");
    return ODF_OK;
}

}  // extern "C"
