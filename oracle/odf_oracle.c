/*
 * odf_oracle.c -- plain FP64 CPU oracle for order-statistics directional
 * filters (Celebi, "Real-time implementation of order-statistics based
 * directional filters", arXiv:1009.0958).
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load this library.  It
 * shares no code, header, table or helper with the GPU library: every
 * definition below is written out again from the paper.
 *
 * Everything is evaluated in IEEE double precision, one window at a time,
 * with the n^2 pair terms of every window computed directly (no reuse of
 * pair terms between windows, no box sums).  No fast-math.
 *
 * Notation (Section II): an M x N RGB image, a sqrt(n) x sqrt(n) window
 * W(r,c) centred on (r,c), members re-indexed i = 1..n.  Here members are
 * numbered u = 0..n-1 in row-major order inside the window, so the centre is
 * u = (n-1)/2, the 0-based form of d = (n+1)/2 in eq. (9).
 *
 * Readings of points the paper leaves open (each one is also listed with the
 * tests that pin it):
 *   - border: windows take replicated (clamped) border pixels, so every
 *     window has n members;
 *   - ties: the lowest member index wins;
 *   - zero vectors: the direction of x = 0 is taken as (1,1,1) for the angle
 *     (eq. 2), the minimax angle (eqs. 4-6) and the chromaticity (eq. 7); the
 *     Minkowski distance uses the true value;
 *   - the direction of a pixel of non-negative integers is x / gcd(x), the
 *     same for every positive multiple of a colour (those terms are
 *     scale-free), so collinear colours tie exactly and the lowest index wins;
 *   - DDF weighting: Omega = A^(1-p) * D^p (p = 1/2 orders the windows as the
 *     product of eq. 3 does), with C pow semantics (0^0 = 1);
 *   - the angle of eq. (2) is evaluated as atan2(|a x b|, a.b), the same
 *     angle, because acos loses accuracy next to 1 (Section 2.1 notes the
 *     ill-conditioning of ACOS near 1);
 *   - minimax (Section 2.1, eqs. 4-6, Table 1): ACOS row in z for z < 1/2,
 *     ASIN row in tau = sqrt(1 - z) for z >= 1/2, the branch decided by the
 *     exact predicate 4 (a.b)^2 < |a|^2 |b|^2, 1 - z formed as
 *     |a x b|^2 / (|a|^2 |b|^2 (1 + z)), and the value clamped at 0 (the q = 3
 *     ASIN row is negative at tau = 0);
 *   - chromaticity distance (Section 2.2, eq. 7) with Minkowski order 2, used
 *     raw by BVDF and through the line of eq. (10) by DDF;
 *   - the self pair j = i is part of every sum, through the same pair
 *     function as every other pair;
 *   - ACWDDF (Section III, Experiment 2): CWDDF^k applies the centre weights
 *     of eq. (9) to both sums of eq. (3); lambda is limited to [1, d - 2] so
 *     that every level k = lambda .. lambda + 2 lies in [1, d];
 *   - the centre-weighted filters on their own: CWVMF^k is eq. (9) with the
 *     Minkowski order p = 2, CWDDF^k the reading above, for k in [1, d].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OK_BVDF = 0, OK_DDF = 1 };
/* members of the largest window, 15 x 15 (the member index is stored in a byte) */
enum { NMAX = 225 };
enum { OD_EXACT = 0, OD_MINIMAX = 1, OD_RGB = 2 };

/* Table 1: minimax polynomial coefficients a_0..a_4 as printed, rows q = 2,3,4. */
static const double TAB1_ASIN[3][5] = {
    {1.829125e-03, 1.371117, 1.480266e-01, 0.0, 0.0},
    {-1.358425e-04, 1.419488, -3.090315e-02, 1.666491e-01, 0.0},
    {2.097797e-05, 1.412840, 1.429881e-02, 6.704361e-02, 6.909677e-02},
};
static const double TAB1_ACOS[3][5] = {
    {1.569882, -9.695260e-01, -1.480266e-01, 0.0, 0.0},
    {1.570864, -1.003730, 3.090318e-02, -2.356775e-01, 0.0},
    {1.570786, -9.990285e-01, -1.429899e-02, -9.481335e-02, -1.381942e-01},
};

/* eq. (10): A ~= ALPHA * B + BETA. */
static const double EQ10_ALPHA = 1.436437;
static const double EQ10_BETA = 0.027664;

static uint64_t gcd_u64(uint64_t a, uint64_t b) {
    while (b) {
        uint64_t r = a % b;
        a = b;
        b = r;
    }
    return a;
}

/* Direction used by the angle and chromaticity terms (eqs. 2 and 7 depend on
 * a pixel only through its direction): the achromatic axis (1,1,1) when x = 0
 * (both are 0/0 there); for a pixel of non-negative integers (every uint8
 * pixel) the canonical integer direction x / gcd(x0, x1, x2), so that
 * collinear colours of different brightness are one vector and every term
 * they enter is equal bit for bit; otherwise x itself. */
static void direction_of(const double *x, double *d) {
    if (x[0] == 0.0 && x[1] == 0.0 && x[2] == 0.0) {
        d[0] = d[1] = d[2] = 1.0;
        return;
    }
    int integral = 1;
    for (int k = 0; k < 3; ++k)
        integral &= x[k] >= 0.0 && x[k] < 9007199254740992.0 && x[k] == floor(x[k]);
    if (integral) {
        uint64_t g = gcd_u64(gcd_u64((uint64_t)x[0], (uint64_t)x[1]), (uint64_t)x[2]);
        for (int k = 0; k < 3; ++k) d[k] = (double)((uint64_t)x[k] / g);
    } else {
        d[0] = x[0]; d[1] = x[1]; d[2] = x[2];
    }
}

/* eq. (2): the angle between a and b. */
static double angle_exact(const double *a, const double *b) {
    double p[3], q[3];
    direction_of(a, p);
    direction_of(b, q);
    double dot = p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
    double c0 = p[1] * q[2] - p[2] * q[1];
    double c1 = p[2] * q[0] - p[0] * q[2];
    double c2 = p[0] * q[1] - p[1] * q[0];
    double s = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    return atan2(s, dot);
}

/* Horner evaluation of a_0 + a_1 t + ... + a_q t^q (eq. 4). */
static double poly_eval(const double *coef, int q, double t) {
    double acc = coef[q];
    for (int k = q - 1; k >= 0; --k) acc = acc * t + coef[k];
    return acc;
}

/* Section 2.1, Method 1: acos replaced by a degree-q minimax polynomial,
 * with the substitution of eqs. (5)-(6) for z >= 1/2. */
static double angle_minimax(const double *a, const double *b, int q) {
    double p[3], r[3];
    direction_of(a, p);
    direction_of(b, r);
    double dot = p[0] * r[0] + p[1] * r[1] + p[2] * r[2];
    double na2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    double nb2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double z = dot / sqrt(na2 * nb2);
    double v;
    if (dot < 0.0 || 4.0 * dot * dot < na2 * nb2) {
        v = poly_eval(TAB1_ACOS[q - 2], q, z); /* z in [0, 1/2) */
    } else {
        double c0 = p[1] * r[2] - p[2] * r[1];
        double c1 = p[2] * r[0] - p[0] * r[2];
        double c2 = p[0] * r[1] - p[1] * r[0];
        double cross2 = c0 * c0 + c1 * c1 + c2 * c2;
        double one_minus_z = cross2 / (na2 * nb2 * (1.0 + z));
        double tau = sqrt(one_minus_z); /* eq. (6), tau in [0, 1/sqrt 2] */
        v = poly_eval(TAB1_ASIN[q - 2], q, tau);
    }
    return v > 0.0 ? v : 0.0;
}

/* eq. (7): L2 distance between chromaticities x / (x1 + x2 + x3). */
static double chroma_dist(const double *a, const double *b) {
    double p[3], r[3];
    direction_of(a, p);
    direction_of(b, r);
    double sp = p[0] + p[1] + p[2];
    double sr = r[0] + r[1] + r[2];
    double e0 = p[0] / sp - r[0] / sr;
    double e1 = p[1] / sp - r[1] / sr;
    double e2 = p[2] / sp - r[2] / sr;
    return sqrt(e0 * e0 + e1 * e1 + e2 * e2);
}

/* Pair term of the angular ordering for the chosen variant. */
static double pair_term(const double *a, const double *b, int kind, int dist, int q) {
    switch (dist) {
    case OD_EXACT: return angle_exact(a, b);
    case OD_MINIMAX: return angle_minimax(a, b, q);
    default: {
        double B = chroma_dist(a, b);
        /* BVDF uses B raw (Experiment 1); the DDF family plugs B into eq. (10)
         * (Experiment 2). */
        return kind == OK_DDF ? EQ10_ALPHA * B + EQ10_BETA : B;
    }
    }
}

/* eq. (1) with p = 2 (Section III uses the L2 norm): raw values. */
static double minkowski_l2(const double *a, const double *b) {
    double e0 = a[0] - b[0], e1 = a[1] - b[1], e2 = a[2] - b[2];
    return sqrt(e0 * e0 + e1 * e1 + e2 * e2);
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Objective of member u: BVDF (eq. 2) orders by A; DDF by A^(1-p) D^p. */
static double objective(double A, double D, int kind, double p) {
    if (kind == OK_BVDF) return A;
    return pow(A, 1.0 - p) * pow(D, p);
}

/* Window members of pixel (r, c) of image b, row-major, replicated border.
 * Writes n source offsets (flat pixel index) into src. */
static void window_members(int M, int N, int w, int r, int c, int64_t *src) {
    int h = (w - 1) / 2, u = 0;
    for (int dy = -h; dy <= h; ++dy)
        for (int dx = -h; dx <= h; ++dx, ++u)
            src[u] = (int64_t)clampi(r + dy, 0, M - 1) * N + clampi(c + dx, 0, N - 1);
}

/* One window: aggregates, objective, argmin (eqs. 1-3). */
static void filter_one(const double *img, int M, int N, int w, int kind, double p, int dist, int q,
                       int64_t pix, double *out, uint8_t *idx, double *A_out, double *D_out,
                       double *O_out) {
    int64_t mn = (int64_t)M * N;
    int64_t b = pix / mn, rc = pix % mn;
    int r = (int)(rc / N), c = (int)(rc % N);
    int n = w * w;
    int64_t src[NMAX];
    double A[NMAX], D[NMAX], Om[NMAX];
    const double *base = img + b * mn * 3;
    window_members(M, N, w, r, c, src);
    for (int u = 0; u < n; ++u) {
        const double *xu = base + src[u] * 3;
        double a = 0.0, d = 0.0;
        for (int v = 0; v < n; ++v) {
            const double *xv = base + src[v] * 3;
            a += pair_term(xu, xv, kind, dist, q);
            if (kind == OK_DDF) d += minkowski_l2(xu, xv);
        }
        A[u] = a;
        D[u] = d;
        Om[u] = objective(a, d, kind, p);
    }
    int best = 0;
    for (int u = 1; u < n; ++u)
        if (Om[u] < Om[best]) best = u;
    const double *sel = base + src[best] * 3;
    if (out) { out[0] = sel[0]; out[1] = sel[1]; out[2] = sel[2]; }
    if (idx) *idx = (uint8_t)best;
    for (int u = 0; u < n; ++u) {
        if (A_out) A_out[u] = A[u];
        if (D_out) D_out[u] = D[u];
        if (O_out) O_out[u] = Om[u];
    }
}

static int check_args(int B, int M, int N, int w, int kind, double p, int dist, int q) {
    if (B < 1 || M < 1 || N < 1) return -1;
    if (w < 3 || w > 15 || w % 2 == 0) return -1; /* odd sqrt(n) x sqrt(n) windows */
    if (kind != OK_BVDF && kind != OK_DDF) return -1;
    if (dist < OD_EXACT || dist > OD_RGB) return -1;
    if (dist == OD_MINIMAX && (q < 2 || q > 4)) return -1;
    if (kind == OK_DDF && !(p >= 0.0 && p <= 1.0)) return -1;
    return 0;
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* ---------------------------------------------------------------- exports */

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Pair terms of `count` (a, b) pairs: theta[i] = pair term, l2[i] = eq. (1). */
int oracle_pair_terms(const double *a, const double *b, int64_t count, int kind, int dist, int q,
                      double *theta, double *l2) {
    if (check_args(1, 1, 1, 3, kind, 0.5, dist, q)) return -1;
    for (int64_t i = 0; i < count; ++i) {
        if (theta) theta[i] = pair_term(a + 3 * i, b + 3 * i, kind, dist, q);
        if (l2) l2[i] = minkowski_l2(a + 3 * i, b + 3 * i);
    }
    return 0;
}

/* Full filter over a batch of B images, B x M x N x 3 interleaved.
 * out: B x M x N x 3; idx: B x M x N; A, D, Omega: B x M x N x n (each nullable). */
int oracle_filter(const double *img, int B, int M, int N, int w, int kind, double p, int dist,
                  int q, double *out, uint8_t *idx, double *A, double *D, double *Omega,
                  int nthreads) {
    if (check_args(B, M, N, w, kind, p, dist, q) || !img) return -1;
    set_threads(nthreads);
    int64_t total = (int64_t)B * M * N;
    int n = w * w;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t pix = 0; pix < total; ++pix) {
        filter_one(img, M, N, w, kind, p, dist, q, pix, out ? out + 3 * pix : NULL,
                   idx ? idx + pix : NULL, A ? A + n * pix : NULL, D ? D + n * pix : NULL,
                   Omega ? Omega + n * pix : NULL);
    }
    return 0;
}

/* The same filter at a list of flat pixel positions pix[k] = (b*M + r)*N + c;
 * results are packed per listed pixel. */
int oracle_filter_at(const double *img, int B, int M, int N, int w, int kind, double p, int dist,
                     int q, const int64_t *pix, int64_t npix, double *out, uint8_t *idx,
                     double *A, double *D, double *Omega, int nthreads) {
    if (check_args(B, M, N, w, kind, p, dist, q) || !img || (npix > 0 && !pix)) return -1;
    int64_t total = (int64_t)B * M * N;
    for (int64_t k = 0; k < npix; ++k)
        if (pix[k] < 0 || pix[k] >= total) return -1;
    set_threads(nthreads);
    int n = w * w;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < npix; ++k) {
        filter_one(img, M, N, w, kind, p, dist, q, pix[k], out ? out + 3 * k : NULL,
                   idx ? idx + k : NULL, A ? A + n * k : NULL, D ? D + n * k : NULL,
                   Omega ? Omega + n * k : NULL);
    }
    return 0;
}

/* Hard backward of the selection: the upstream gradient of output pixel c
 * goes to the input pixel the window selected, clamp(c + offset(idx(c))).
 * Output pixels are visited in raster order. */
int oracle_backward_hard(const uint8_t *idx, const double *dy, int B, int M, int N, int w,
                         double *dx) {
    if (B < 1 || M < 1 || N < 1 || w < 3 || w > 15 || w % 2 == 0 || !idx || !dy || !dx)
        return -1;
    int h = (w - 1) / 2, n = w * w;
    int64_t mn = (int64_t)M * N;
    memset(dx, 0, sizeof(double) * 3 * mn * B);
    for (int b = 0; b < B; ++b)
        for (int r = 0; r < M; ++r)
            for (int c = 0; c < N; ++c) {
                int64_t pix = b * mn + (int64_t)r * N + c;
                int u = idx[pix];
                if (u >= n) return -1;
                int sr = clampi(r + u / w - h, 0, M - 1), sc = clampi(c + u % w - h, 0, N - 1);
                double *g = dx + 3 * (b * mn + (int64_t)sr * N + sc);
                const double *d = dy + 3 * pix;
                g[0] += d[0]; g[1] += d[1]; g[2] += d[2];
            }
    return 0;
}

/* ------------------------------------------------ softmin relaxation
 * The temperature-tau relaxation of the argmin: member weights
 * pi_u = softmax_u(-(Omega_u - min Omega) / tau) and y = sum_u pi_u x_u.
 * The pair term is the exact angle of eq. (2); DDF adds eq. (1) with p = 2. */

static void softmin_window(const double *base, int M, int N, int w, int kind, double p, double tau,
                           int r, int c, int64_t *src, double *A, double *D, double *Om, double *pi,
                           double *y) {
    int n = w * w;
    window_members(M, N, w, r, c, src);
    for (int u = 0; u < n; ++u) {
        const double *xu = base + src[u] * 3;
        double a = 0.0, d = 0.0;
        for (int v = 0; v < n; ++v) {
            const double *xv = base + src[v] * 3;
            a += angle_exact(xu, xv);
            if (kind == OK_DDF) d += minkowski_l2(xu, xv);
        }
        A[u] = a;
        D[u] = d;
        Om[u] = objective(a, d, kind, p);
    }
    double omin = Om[0];
    for (int u = 1; u < n; ++u)
        if (Om[u] < omin) omin = Om[u];
    double z = 0.0;
    for (int u = 0; u < n; ++u) {
        pi[u] = exp(-(Om[u] - omin) / tau);
        z += pi[u];
    }
    y[0] = y[1] = y[2] = 0.0;
    for (int u = 0; u < n; ++u) {
        pi[u] /= z;
        const double *xu = base + src[u] * 3;
        y[0] += pi[u] * xu[0];
        y[1] += pi[u] * xu[1];
        y[2] += pi[u] * xu[2];
    }
}

int oracle_softmin_fwd(const double *img, int B, int M, int N, int w, int kind, double p,
                       double tau, double *y, double *pi_out, int nthreads) {
    if (check_args(B, M, N, w, kind, p, OD_EXACT, 4) || !(tau > 0.0) || !img || !y) return -1;
    set_threads(nthreads);
    int64_t mn = (int64_t)M * N, total = mn * B;
    int n = w * w;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t pix = 0; pix < total; ++pix) {
        int64_t src[NMAX];
        double A[NMAX], D[NMAX], Om[NMAX], pi[NMAX];
        int64_t b = pix / mn, rc = pix % mn;
        softmin_window(img + b * mn * 3, M, N, w, kind, p, tau, (int)(rc / N), (int)(rc % N), src,
                       A, D, Om, pi, y + 3 * pix);
        if (pi_out)
            for (int u = 0; u < n; ++u) pi_out[n * pix + u] = pi[u];
    }
    return 0;
}

/* Gradient of the angle with respect to its first argument:
 * d theta / d a = -(b^ - cos(theta) a^) / (|a| sin(theta)), taken as 0 where
 * sin(theta) = 0; the direction of the zero vector is a constant, so its
 * gradient is 0. */
static void angle_grad_a(const double *a, const double *b, double *g) {
    g[0] = g[1] = g[2] = 0.0;
    if (a[0] == 0.0 && a[1] == 0.0 && a[2] == 0.0) return;
    double q[3];
    direction_of(b, q);
    double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    double nb = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    double c0 = a[1] * q[2] - a[2] * q[1];
    double c1 = a[2] * q[0] - a[0] * q[2];
    double c2 = a[0] * q[1] - a[1] * q[0];
    double s = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    double dot = a[0] * q[0] + a[1] * q[1] + a[2] * q[2];
    double sn = s / (na * nb), cs = dot / (na * nb); /* sin and cos of the angle */
    if (sn == 0.0) return;
    for (int k = 0; k < 3; ++k) g[k] = -(q[k] / nb - cs * a[k] / na) / (na * sn);
}

/* Gradient of |a - b| with respect to a: (a - b)/|a - b|, 0 where a = b. */
static void l2_grad_a(const double *a, const double *b, double *g) {
    double e0 = a[0] - b[0], e1 = a[1] - b[1], e2 = a[2] - b[2];
    double l = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    if (l == 0.0) { g[0] = g[1] = g[2] = 0.0; return; }
    g[0] = e0 / l; g[1] = e1 / l; g[2] = e2 / l;
}

/* Partial derivatives of Omega = A^(1-p) D^p, each taken as 0 where its
 * aggregate is 0 and the power is fractional. */
static void objective_grad(double A, double D, double Om, int kind, double p, double *dA, double *dD) {
    if (kind == OK_BVDF || p == 0.0) { *dA = 1.0; *dD = 0.0; return; }
    if (p == 1.0) { *dA = 0.0; *dD = 1.0; return; }
    *dA = A > 0.0 ? (1.0 - p) * Om / A : 0.0;
    *dD = D > 0.0 ? p * Om / D : 0.0;
}

/* Reverse mode of the softmin relaxation, written out from the chain rule:
 * y = sum_u pi_u x_u, pi = softmax(-Omega / tau), Omega_u = Omega(A_u, D_u),
 * A_u = sum_v theta(x_u, x_v), D_u = sum_v |x_u - x_v|.  Every contribution is
 * added into the source pixel the member was read from.  Images are
 * processed in parallel; inside an image, output pixels in raster order. */
int oracle_softmin_bwd(const double *img, const double *dy, int B, int M, int N, int w, int kind,
                       double p, double tau, double *dx, int nthreads) {
    if (check_args(B, M, N, w, kind, p, OD_EXACT, 4) || !(tau > 0.0) || !img || !dy || !dx)
        return -1;
    set_threads(nthreads);
    int64_t mn = (int64_t)M * N;
    int n = w * w;
    memset(dx, 0, sizeof(double) * 3 * mn * B);
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < B; ++b) {
        const double *base = img + (int64_t)b * mn * 3;
        double *gx = dx + (int64_t)b * mn * 3;
        for (int64_t rc = 0; rc < mn; ++rc) {
            int64_t src[NMAX];
            double A[NMAX], D[NMAX], Om[NMAX], pi[NMAX], y[3];
            softmin_window(base, M, N, w, kind, p, tau, (int)(rc / N), (int)(rc % N), src, A, D,
                           Om, pi, y);
            const double *g = dy + 3 * ((int64_t)b * mn + rc);
            for (int u = 0; u < n; ++u) {
                const double *xu = base + src[u] * 3;
                /* direct path: dy/dx_u = pi_u I */
                double *t = gx + src[u] * 3;
                t[0] += pi[u] * g[0]; t[1] += pi[u] * g[1]; t[2] += pi[u] * g[2];
                /* through the weights: d y / d Omega_u = -pi_u (x_u - y) / tau */
                double gom = -pi[u] *
                             ((xu[0] - y[0]) * g[0] + (xu[1] - y[1]) * g[1] + (xu[2] - y[2]) * g[2]) /
                             tau;
                double dA, dD;
                objective_grad(A[u], D[u], Om[u], kind, p, &dA, &dD);
                double gA = gom * dA, gD = gom * dD;
                for (int v = 0; v < n; ++v) {
                    const double *xv = base + src[v] * 3;
                    double ga[3], gb[3];
                    double *su = gx + src[u] * 3, *sv = gx + src[v] * 3;
                    if (gA != 0.0) {
                        angle_grad_a(xu, xv, ga);
                        angle_grad_a(xv, xu, gb);
                        for (int k = 0; k < 3; ++k) { su[k] += gA * ga[k]; sv[k] += gA * gb[k]; }
                    }
                    if (gD != 0.0) {
                        l2_grad_a(xu, xv, ga);
                        for (int k = 0; k < 3; ++k) { su[k] += gD * ga[k]; sv[k] -= gD * ga[k]; }
                    }
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------- ACWDDF
 * Adaptive centre-weighted directional distance filter (Section III,
 * Experiment 2: the switching rule and eq. 9).
 *
 * Weights of eq. (9): w_v(k) = n - 2k + 2 for the window centre v = d and 1
 * for every other member, smoothing level k in [1, d], d = (n + 1) / 2
 * (1-based; the centre is member (n - 1) / 2 here).
 *
 * CWDDF^k (reading: the rule names CWDDF^k but eq. 9 writes out only the
 * centre-weighted VMF): the weights of eq. (9) applied to both sums of eq. (3),
 *   Omega^k_u = (sum_v w_v(k) A(x_u, x_v)) * (sum_v w_v(k) L2(x_u, x_v)),
 * and y_CWDDF^k the member of lowest index with the smallest Omega^k.
 *
 * Switch: S = sum_{k = lambda}^{lambda + 2} A(y_CWDDF^k, x_d) * L2(y_CWDDF^k, x_d).
 * The output is the DDF output (eq. 3, the plain product) when S > T and the
 * centre x_d otherwise.  k must stay in [1, d], so lambda is taken in
 * [1, d - 2] (the rule's lambda in [1, d - 1] would reach k = d + 1).
 * A(.,.) is the variant's pair term: the exact angle, the minimax angle of
 * Method 1, or eq. (10) applied to the chromaticity distance of Method 2.
 *
 * diag (nullable, 5n doubles per pixel): [0, n) Omega of eq. (3); then
 * Omega^k for k = lambda, lambda + 1, lambda + 2 (n each); then
 * A(x_u, x_d) * L2(x_u, x_d) for every member u. */
static void acwddf_one(const double *img, int M, int N, int w, int dist, int q, int lambda,
                       double T, int64_t pix, double *out, uint8_t *idx, double *S_out,
                       double *diag) {
    int64_t mn = (int64_t)M * N;
    int64_t b = pix / mn, rc = pix % mn;
    int r = (int)(rc / N), c = (int)(rc % N);
    int n = w * w, d = (n - 1) / 2;
    int64_t src[NMAX];
    double Om[4][NMAX];
    /* the n x n pair terms of the window, th[u n + v] and l2[u n + v] (on the
     * heap: 810 KB at 15 x 15) */
    double *th = malloc(sizeof(double) * n * n), *l2 = malloc(sizeof(double) * n * n);
    if (!th || !l2) abort();
    const double *base = img + b * mn * 3;
    window_members(M, N, w, r, c, src);
    for (int u = 0; u < n; ++u)
        for (int v = 0; v < n; ++v) {
            th[u * n + v] = pair_term(base + src[u] * 3, base + src[v] * 3, OK_DDF, dist, q);
            l2[u * n + v] = minkowski_l2(base + src[u] * 3, base + src[v] * 3);
        }
    /* eq. (3) and the three centre-weighted objectives */
    for (int j = 0; j < 4; ++j) {
        int k = lambda + j - 1;
        for (int u = 0; u < n; ++u) {
            double a = 0.0, e = 0.0;
            for (int v = 0; v < n; ++v) {
                double wv = (j > 0 && v == d) ? (double)(n - 2 * k + 2) : 1.0;
                a += wv * th[u * n + v];
                e += wv * l2[u * n + v];
            }
            Om[j][u] = a * e;
        }
    }
    int sel[4];
    for (int j = 0; j < 4; ++j) {
        sel[j] = 0;
        for (int u = 1; u < n; ++u)
            if (Om[j][u] < Om[j][sel[j]]) sel[j] = u;
    }
    double S = 0.0;
    for (int j = 1; j < 4; ++j) S += th[sel[j] * n + d] * l2[sel[j] * n + d];
    int chosen = S > T ? sel[0] : d;
    const double *x = base + src[chosen] * 3;
    if (out) { out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; }
    if (idx) *idx = (uint8_t)chosen;
    if (S_out) *S_out = S;
    if (diag) {
        for (int j = 0; j < 4; ++j)
            for (int u = 0; u < n; ++u) diag[j * n + u] = Om[j][u];
        for (int u = 0; u < n; ++u) diag[4 * n + u] = th[u * n + d] * l2[u * n + d];
    }
    free(th);
    free(l2);
}

static int check_acw(int B, int M, int N, int w, int dist, int q, int lambda, double T) {
    if (check_args(B, M, N, w, OK_DDF, 0.5, dist, q)) return -1;
    int dd = (w * w + 1) / 2;
    if (lambda < 1 || lambda > dd - 2 || T != T) return -1;
    return 0;
}

/* Full ACWDDF over B images; out B x M x N x 3, idx and S B x M x N, diag
 * B x M x N x 5n (each nullable). */
int oracle_acwddf(const double *img, int B, int M, int N, int w, int dist, int q, int lambda,
                  double T, double *out, uint8_t *idx, double *S, double *diag, int nthreads) {
    if (check_acw(B, M, N, w, dist, q, lambda, T) || !img) return -1;
    set_threads(nthreads);
    int64_t total = (int64_t)B * M * N;
    int n = w * w;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t pix = 0; pix < total; ++pix)
        acwddf_one(img, M, N, w, dist, q, lambda, T, pix, out ? out + 3 * pix : NULL,
                   idx ? idx + pix : NULL, S ? S + pix : NULL, diag ? diag + 5 * n * pix : NULL);
    return 0;
}

/* ACWDDF at listed flat pixel positions; results packed per listed pixel. */
int oracle_acwddf_at(const double *img, int B, int M, int N, int w, int dist, int q, int lambda,
                     double T, const int64_t *pix, int64_t npix, double *out, uint8_t *idx,
                     double *S, double *diag, int nthreads) {
    if (check_acw(B, M, N, w, dist, q, lambda, T) || !img || (npix > 0 && !pix)) return -1;
    int64_t total = (int64_t)B * M * N;
    for (int64_t k = 0; k < npix; ++k)
        if (pix[k] < 0 || pix[k] >= total) return -1;
    set_threads(nthreads);
    int n = w * w;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < npix; ++k)
        acwddf_one(img, M, N, w, dist, q, lambda, T, pix[k], out ? out + 3 * k : NULL,
                   idx ? idx + k : NULL, S ? S + k : NULL, diag ? diag + 5 * n * k : NULL);
    return 0;
}

/* ------------------------------------------------ centre-weighted filters
 * CWVMF^k (eq. 9): the member minimising sum_v w_v(k) L2(x_u, x_v), with
 * w_d(k) = n - 2k + 2 on the centre member and 1 elsewhere, k in [1, d].
 * CWDDF^k: the same weights on both sums of eq. (3), the member minimising
 * (sum_v w_v(k) A(x_u, x_v)) * (sum_v w_v(k) L2(x_u, x_v)), A the variant's
 * pair term as in ACWDDF (eq. 10 on the chromaticity distance for Method 2).
 * obj (nullable, n doubles per pixel): the objective of every member. */
static void cw_one(const double *img, int M, int N, int w, int vmf, int dist, int q, int level,
                   int64_t pix, double *out, uint8_t *idx, double *obj) {
    int64_t mn = (int64_t)M * N;
    int64_t b = pix / mn, rc = pix % mn;
    int r = (int)(rc / N), c = (int)(rc % N);
    int n = w * w, d = (n - 1) / 2;
    int64_t src[NMAX];
    double Om[NMAX];
    const double *base = img + b * mn * 3;
    window_members(M, N, w, r, c, src);
    for (int u = 0; u < n; ++u) {
        double a = 0.0, e = 0.0;
        for (int v = 0; v < n; ++v) {
            double wv = v == d ? (double)(n - 2 * level + 2) : 1.0;
            const double *xu = base + src[u] * 3, *xv = base + src[v] * 3;
            if (!vmf) a += wv * pair_term(xu, xv, OK_DDF, dist, q);
            e += wv * minkowski_l2(xu, xv);
        }
        Om[u] = vmf ? e : a * e;
    }
    int sel = 0;
    for (int u = 1; u < n; ++u)
        if (Om[u] < Om[sel]) sel = u;
    const double *x = base + src[sel] * 3;
    if (out) { out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; }
    if (idx) *idx = (uint8_t)sel;
    if (obj)
        for (int u = 0; u < n; ++u) obj[u] = Om[u];
}

/* CWVMF^k (vmf = 1) or CWDDF^k (vmf = 0) over B images; out, idx, obj nullable. */
int oracle_cwfilter(const double *img, int B, int M, int N, int w, int vmf, int dist, int q,
                    int level, double *out, uint8_t *idx, double *obj, int nthreads) {
    if (check_args(B, M, N, w, OK_DDF, 0.5, dist, q) || !img) return -1;
    if (level < 1 || level > (w * w + 1) / 2 || (vmf != 0 && vmf != 1)) return -1;
    set_threads(nthreads);
    int64_t total = (int64_t)B * M * N;
    int n = w * w;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t pix = 0; pix < total; ++pix)
        cw_one(img, M, N, w, vmf, dist, q, level, pix, out ? out + 3 * pix : NULL,
               idx ? idx + pix : NULL, obj ? obj + (int64_t)n * pix : NULL);
    return 0;
}
