// softmin64.hip -- binary64 twins of the softmin relaxation and of its
// gradient, for gradient checks by finite differences in binary64.
//
// Written from the definitions, not for speed: one thread per window forms
// its n members (replicated border), every pair term directly (the exact angle
// of eq. 2 as atan2(|a x b|, a . b) on the directions, the L2 distance on the
// raw values), the aggregates A and D, the objective Omega = A^(1-p) D^p
// (eq. 3 generalised; BVDF Omega = A), the weights
// pi_u = exp(-(Omega_u - min Omega) / tau) / Z and y = sum_u pi_u x_u.  No
// tiles, no reuse of pair terms between windows.
//
// Backward (chain rule, per window c): with s_u = dy(c) . (x_u - y),
//   dL/dOmega_u = -pi_u s_u / tau,
//   dL/dA_u = dL/dOmega_u dOmega/dA, dL/dD_u = dL/dOmega_u dOmega/dD,
// and, as the pair term of (u, v) enters both A_u and A_v,
//   g_u(c) = pi_u dy(c) + sum_{v != u} (dL/dA_u + dL/dA_v) dtheta(u, v)/dx_u
//                       + sum_{v != u} (dL/dD_u + dL/dD_v) dL2(u, v)/dx_u,
// dtheta/da = -(b^ - cos(theta) a^) / (|a| sin(theta)) (0 where sin(theta) = 0,
// and 0 for a zero pixel, whose direction is the constant (1, 1, 1)),
// dL2/da = (a - b) / |a - b| (0 where a = b).  dOmega/dA = 1 and dOmega/dD = 0
// for BVDF and p = 0, the reverse for p = 1, else (1 - p) Omega / A and
// p Omega / D, each 0 where its aggregate is 0.  A first kernel writes g_u(c)
// for every window and member to the workspace; a second gathers, for every
// pixel q, the g_u(c) of the members that are q (windows c in raster order,
// u ascending), so the result does not depend on scheduling.
#include <math.h>

#include "odf.h"
#include "odf_internal.h"

// No contraction into fused multiply-adds: the cross product of two equal
// directions (a member and its copy at the replicated border) must come out
// exactly 0, so that the angle gradient of the pair is the defined 0 rather
// than the rounding residue of ab - cd over a near-zero sine.
#pragma clang fp contract(off)

namespace odf {
namespace {

struct Soft64Params {
    const double* x;   // B x M x N x 3
    const double* dy;  // backward: upstream gradient
    double* y;         // forward output
    double* g;         // backward: B x M x N x n x 3 per-window member gradients
    double* dx;        // backward output
    int B, M, N;
    int ddf;           // 0: BVDF (Omega = A), 1: DDF
    double p, tau;
};

constexpr int kSoft64Threads = 256;

__device__ inline void direction(const double (&x)[3], double (&d)[3]) {
    const bool zero = x[0] == 0.0 && x[1] == 0.0 && x[2] == 0.0;
    for (int k = 0; k < 3; ++k) d[k] = zero ? 1.0 : x[k];
}

__device__ inline double pair_angle(const double (&a)[3], const double (&b)[3]) {
    double da[3], db[3];
    direction(a, da);
    direction(b, db);
    const double c0 = da[1] * db[2] - da[2] * db[1];
    const double c1 = da[2] * db[0] - da[0] * db[2];
    const double c2 = da[0] * db[1] - da[1] * db[0];
    return atan2(sqrt(c0 * c0 + c1 * c1 + c2 * c2), da[0] * db[0] + da[1] * db[1] + da[2] * db[2]);
}

__device__ inline double pair_l2(const double (&a)[3], const double (&b)[3]) {
    const double e0 = a[0] - b[0], e1 = a[1] - b[1], e2 = a[2] - b[2];
    return sqrt(e0 * e0 + e1 * e1 + e2 * e2);
}

// dtheta(a, b)/da (0 for parallel directions and for the zero pixel a)
__device__ inline void angle_grad(const double (&a)[3], const double (&b)[3], double (&g)[3]) {
    g[0] = g[1] = g[2] = 0.0;
    if (a[0] == 0.0 && a[1] == 0.0 && a[2] == 0.0) return;
    double db[3];
    direction(b, db);
    const double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    const double nb = sqrt(db[0] * db[0] + db[1] * db[1] + db[2] * db[2]);
    double ah[3], bh[3];
    for (int k = 0; k < 3; ++k) {
        ah[k] = a[k] / na;
        bh[k] = db[k] / nb;
    }
    const double c0 = ah[1] * bh[2] - ah[2] * bh[1];
    const double c1 = ah[2] * bh[0] - ah[0] * bh[2];
    const double c2 = ah[0] * bh[1] - ah[1] * bh[0];
    const double s = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    if (s == 0.0) return;
    const double c = ah[0] * bh[0] + ah[1] * bh[1] + ah[2] * bh[2];
    for (int k = 0; k < 3; ++k) g[k] = -(bh[k] - c * ah[k]) / (na * s);
}

__device__ inline void objective_grad64(const Soft64Params& prm, double A, double D, double Om,
                                        double& dA, double& dD) {
    if (!prm.ddf || prm.p == 0.0) {
        dA = 1.0;
        dD = 0.0;
    } else if (prm.p == 1.0) {
        dA = 0.0;
        dD = 1.0;
    } else {
        dA = A > 0.0 ? (1.0 - prm.p) * Om / A : 0.0;
        dD = D > 0.0 ? prm.p * Om / D : 0.0;
    }
}

// One window per thread: the forward output, or (BWD) the gradient of every
// member of the window.
template <int W, bool BWD>
__global__ void __launch_bounds__(kSoft64Threads) soft64_window(Soft64Params prm) {
    constexpr int H = W / 2, NW = W * W;
    const int M = prm.M, N = prm.N;
    const int npix = prm.B * M * N;  // < 2^31, checked on the host
    const int blk = flat_block((npix + kSoft64Threads - 1) / kSoft64Threads);
    if (blk < 0) return;
    const int c = blk * kSoft64Threads + (int)threadIdx.x;
    if (c >= npix) return;
    const int b = c / (M * N), r = (c / N) % M, col = c % N;

    double xm[NW][3];
#pragma unroll 1
    for (int u = 0; u < NW; ++u) {
        const int ry = min(max(r + u / W - H, 0), M - 1);
        const int rx = min(max(col + u % W - H, 0), N - 1);
        const double* s = prm.x + ((size_t)(b * M + ry) * N + rx) * 3;
        for (int k = 0; k < 3; ++k) xm[u][k] = s[k];
    }
    double A[NW], D[NW], Om[NW], pi[NW];
    double om_min = 0.0;
#pragma unroll 1
    for (int u = 0; u < NW; ++u) {
        double a = 0.0, d = 0.0;
#pragma unroll 1
        for (int v = 0; v < NW; ++v) {
            a += pair_angle(xm[u], xm[v]);
            if (prm.ddf) d += pair_l2(xm[u], xm[v]);
        }
        A[u] = a;
        D[u] = d;
        Om[u] = prm.ddf ? pow(a, 1.0 - prm.p) * pow(d, prm.p) : a;
        om_min = u == 0 ? Om[u] : fmin(om_min, Om[u]);
    }
    double z = 0.0;
#pragma unroll 1
    for (int u = 0; u < NW; ++u) {
        pi[u] = exp(-(Om[u] - om_min) / prm.tau);
        z += pi[u];
    }
    double y[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
    for (int u = 0; u < NW; ++u) {
        pi[u] /= z;
        for (int k = 0; k < 3; ++k) y[k] += pi[u] * xm[u][k];
    }
    if (!BWD) {
        for (int k = 0; k < 3; ++k) prm.y[(size_t)c * 3 + k] = y[k];
        return;
    }
    const double* dyc = prm.dy + (size_t)c * 3;
    const double g0 = dyc[0], g1 = dyc[1], g2 = dyc[2];
    double gA[NW], gD[NW];
#pragma unroll 1
    for (int u = 0; u < NW; ++u) {
        const double s = g0 * (xm[u][0] - y[0]) + g1 * (xm[u][1] - y[1]) + g2 * (xm[u][2] - y[2]);
        const double gom = -pi[u] * s / prm.tau;
        double dA, dD;
        objective_grad64(prm, A[u], D[u], Om[u], dA, dD);
        gA[u] = gom * dA;
        gD[u] = gom * dD;
    }
#pragma unroll 1
    for (int u = 0; u < NW; ++u) {
        double acc[3] = {pi[u] * g0, pi[u] * g1, pi[u] * g2};
#pragma unroll 1
        for (int v = 0; v < NW; ++v) {
            if (v == u) continue;
            const double ct = gA[u] + gA[v];
            if (ct != 0.0) {
                double ga[3];
                angle_grad(xm[u], xm[v], ga);
                for (int k = 0; k < 3; ++k) acc[k] += ct * ga[k];
            }
            const double cl = gD[u] + gD[v];
            const double l = pair_l2(xm[u], xm[v]);
            if (cl != 0.0 && l > 0.0)
                for (int k = 0; k < 3; ++k) acc[k] += cl * (xm[u][k] - xm[v][k]) / l;
        }
        double* o = prm.g + ((size_t)c * NW + u) * 3;
        for (int k = 0; k < 3; ++k) o[k] = acc[k];
    }
}

// dx(q): the member gradients of every window member that is the pixel q
// (within h of q, replicated border), windows in raster order, members in
// index order.
template <int W>
__global__ void __launch_bounds__(kSoft64Threads) soft64_gather(Soft64Params prm) {
    constexpr int H = W / 2, NW = W * W;
    const int M = prm.M, N = prm.N;
    const int npix = prm.B * M * N;
    const int blk = flat_block((npix + kSoft64Threads - 1) / kSoft64Threads);
    if (blk < 0) return;
    const int q = blk * kSoft64Threads + (int)threadIdx.x;
    if (q >= npix) return;
    const int b = q / (M * N), qy = (q / N) % M, qx = q % N;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int cy = max(qy - H, 0); cy <= min(qy + H, M - 1); ++cy)
        for (int cx = max(qx - H, 0); cx <= min(qx + H, N - 1); ++cx) {
            const size_t c = (size_t)(b * M + cy) * N + cx;
            for (int u = 0; u < NW; ++u) {
                if (min(max(cy + u / W - H, 0), M - 1) != qy ||
                    min(max(cx + u % W - H, 0), N - 1) != qx)
                    continue;
                const double* g = prm.g + (c * NW + u) * 3;
                for (int k = 0; k < 3; ++k) acc[k] += g[k];
            }
        }
    for (int k = 0; k < 3; ++k) prm.dx[(size_t)q * 3 + k] = acc[k];
}

template <int W>
hipError_t launch_soft64_w(bool bwd, const Soft64Params& prm, hipStream_t s) {
    const long long npix = (long long)prm.B * prm.M * prm.N;
    const dim3 grid = flat_grid((npix + kSoft64Threads - 1) / kSoft64Threads);
    if (!bwd) {
        hipLaunchKernelGGL((soft64_window<W, false>), grid, dim3(kSoft64Threads), 0, s, prm);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((soft64_window<W, true>), grid, dim3(kSoft64Threads), 0, s, prm);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((soft64_gather<W>), grid, dim3(kSoft64Threads), 0, s, prm);
    return hipGetLastError();
}

bool overlap64(const void* a, size_t na, const void* b, size_t nb) {
    const char* x = static_cast<const char*>(a);
    const char* y = static_cast<const char*>(b);
    return x < y + nb && y < x + na;
}

int check_soft64(const double* x, int B, int M, int N, int window, int kind, double p, double tau) {
    if (!x) return set_error(ODF_EINVAL, "x is NULL");
    if (B < 1 || M < 1 || N < 1)
        return set_error(ODF_EINVAL, "sizes must be >= 1 (B=%d M=%d N=%d)", B, M, N);
    if ((long long)B * M * N >= (1ll << 31)) return set_error(ODF_EINVAL, "B*M*N must be < 2^31 pixels");
    if (window != 3 && window != 5 && window != 7 && window != 9)
        return set_error(ODF_EUNSUPPORTED, "the softmin relaxation supports windows 3 to 9");
    if (kind != ODF_BVDF && kind != ODF_DDF) return set_error(ODF_EINVAL, "kind %d out of range", kind);
    if (kind == ODF_DDF && !(p >= 0.0 && p <= 1.0)) return set_error(ODF_EINVAL, "p must be in [0, 1]");
    if (!(tau > 0.0) || !(tau < 1.0e300)) return set_error(ODF_EINVAL, "tau must be positive and finite");
    return ODF_OK;
}

}  // namespace
}  // namespace odf

extern "C" {

int odf_softmin_fwd_f64(const double* x, int B, int M, int N, int window, int kind, double p,
                        double tau, double* y, void* stream) {
    int rc = odf::check_soft64(x, B, M, N, window, kind, p, tau);
    if (rc) return rc;
    if (!y) return odf::set_error(ODF_EINVAL, "y is NULL");
    const size_t nb = (size_t)B * M * N * 3 * sizeof(double);
    if (odf::overlap64(x, nb, y, nb)) return odf::set_error(ODF_EINVAL, "y overlaps x");
    odf::Soft64Params prm{};
    prm.x = x; prm.y = y; prm.B = B; prm.M = M; prm.N = N;
    prm.ddf = kind == ODF_DDF;
    prm.p = kind == ODF_DDF ? p : 0.0;
    prm.tau = tau;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e = window == 3   ? odf::launch_soft64_w<3>(false, prm, s)
                         : window == 5 ? odf::launch_soft64_w<5>(false, prm, s)
                         : window == 7 ? odf::launch_soft64_w<7>(false, prm, s)
                                       : odf::launch_soft64_w<9>(false, prm, s);
    if (e != hipSuccess)
        return odf::set_error(ODF_EHIP, "binary64 softmin forward launch: %s", hipGetErrorString(e));
    return ODF_OK;
}

size_t odf_softmin_bwd_f64_workspace(int B, int M, int N, int window) {
    if (B < 1 || M < 1 || N < 1 || (long long)B * M * N >= (1ll << 31) ||
        (window != 3 && window != 5 && window != 7 && window != 9))
        return 0;
    return (size_t)B * M * N * window * window * 3 * sizeof(double);
}

int odf_softmin_bwd_f64(const double* x, const double* dy, int B, int M, int N, int window, int kind,
                        double p, double tau, double* dx, void* workspace, size_t workspace_bytes,
                        void* stream) {
    int rc = odf::check_soft64(x, B, M, N, window, kind, p, tau);
    if (rc) return rc;
    if (!dy || !dx || !workspace)
        return odf::set_error(ODF_EINVAL, "dy, dx and workspace must be non-NULL");
    const size_t need = odf_softmin_bwd_f64_workspace(B, M, N, window);
    if (workspace_bytes < need)
        return odf::set_error(ODF_EINVAL, "workspace too small (%zu < %zu bytes)", workspace_bytes,
                              need);
    if ((reinterpret_cast<uintptr_t>(workspace) & 7) != 0)
        return odf::set_error(ODF_EINVAL, "workspace must be 8-byte aligned");
    const size_t nb = (size_t)B * M * N * 3 * sizeof(double);
    if (odf::overlap64(dx, nb, x, nb) || odf::overlap64(dx, nb, dy, nb) ||
        odf::overlap64(workspace, need, x, nb) || odf::overlap64(workspace, need, dy, nb) ||
        odf::overlap64(workspace, need, dx, nb))
        return odf::set_error(ODF_EINVAL, "dx / workspace overlap an input or each other");
    odf::Soft64Params prm{};
    prm.x = x; prm.dy = dy; prm.dx = dx; prm.g = static_cast<double*>(workspace);
    prm.B = B; prm.M = M; prm.N = N;
    prm.ddf = kind == ODF_DDF;
    prm.p = kind == ODF_DDF ? p : 0.0;
    prm.tau = tau;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const hipError_t e = window == 3   ? odf::launch_soft64_w<3>(true, prm, s)
                         : window == 5 ? odf::launch_soft64_w<5>(true, prm, s)
                         : window == 7 ? odf::launch_soft64_w<7>(true, prm, s)
                                       : odf::launch_soft64_w<9>(true, prm, s);
    if (e != hipSuccess)
        return odf::set_error(ODF_EHIP, "binary64 softmin backward launch: %s", hipGetErrorString(e));
    return ODF_OK;
}

}  // extern "C"
