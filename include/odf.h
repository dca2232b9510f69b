/*
 * odf.h -- C ABI of libodf, order-statistics directional vector filters
 * (BVDF, DDF) on AMD Instinct MI355X (gfx950).
 *
 * Method: M. E. Celebi, "Real-time implementation of order-statistics based
 * directional filters", arXiv:1009.0958.
 *
 * Every image is an RGB array in HWC order: pixel (b, r, c) channel k lives at
 * element ((b*M + r)*N + c)*3 + k.  A window of w x w pixels (w = 3, 5, 7 or 9) is
 * centred on each pixel; border windows repeat the nearest edge pixel
 * (replicated border), so every window has n = w*w members.  Members are
 * numbered u = 0..n-1 row-major inside the window; the centre is (n-1)/2.
 *
 * Conventions shared by every entry point:
 *   - All data pointers are DEVICE pointers owned by the caller.  The library
 *     neither frees nor retains them.  Outputs must not overlap inputs.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue work
 *     on it and return without waiting; they allocate nothing except where
 *     stated (odf_batch_plan, the autotuners, odf_tune_load).
 *   - Arguments are validated on the host before anything is launched.  A
 *     rejected call returns a negative odf_status, launches nothing and sets
 *     the message returned by odf_last_error() (per thread).
 *   - Sizes: B, M, N >= 1 and B*M*N < 2^31 pixels per call.
 *   - No C++ exception crosses this interface.
 *   - Tests can make the allocating calls (odf_batch_plan, odf_autotune,
 *     odf_autotune_batch, odf_autotune_batch_jobs) take
 *     their allocation-failure path: with the environment variable
 *     ODF_TEST_FAIL_ALLOC set to anything but "" or "0" they return
 *     ODF_ENOMEM before allocating or touching the device.
 */
#ifndef ODF_H
#define ODF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ODF_OK = 0,
    ODF_EINVAL = -1,        /* bad argument (null pointer, size, range, aliasing) */
    ODF_EUNSUPPORTED = -2,  /* valid request this build does not provide (e.g. w = 9) */
    ODF_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
    ODF_ENOMEM = -4         /* a library-side allocation failed */
} odf_status;

/* Filter family.  BVDF (Section II, eq. 2): member minimising the sum of
 * angles to all window members.  DDF: member minimising
 * Omega_u = A_u^(1-p) * D_u^p, A_u the angle sum of eq. (2) and D_u the sum of
 * L2 distances of eq. (1); p = 1/2 orders members as the product of eq. (3),
 * p = 0 is BVDF and p = 1 the vector median of eq. (1). */
typedef enum {
    ODF_BVDF = 0,
    ODF_DDF = 1,
    ODF_ACWDDF = 2,
    ODF_CWVMF = 3,
    ODF_CWDDF = 4
} odf_kind;
/* ODF_ACWDDF (the adaptive centre-weighted DDF of Section III, Experiment 2)
 * is computed by odf_acwddf_u8 / odf_acwddf_f32 and is accepted as a kind by
 * the tuning calls; ODF_CWVMF and ODF_CWDDF (its centre-weighted levels as
 * filters of their own) by odf_cw_filter_u8 / odf_cw_filter_f32 only.  The
 * other entry points take ODF_BVDF or ODF_DDF. */

/* Angular pair term.  EXACT: the angle of eq. (2).  MINIMAX: Section 2.1
 * (Method 1), the degree-q minimax polynomials of Table 1 with the
 * substitution of eqs. (5)-(6) for cosines >= 1/2.  RGB: Section 2.2
 * (Method 2), the L2 distance between chromaticities (eq. 7); DDF maps it
 * through the line of eq. (10). */
typedef enum { ODF_EXACT = 0, ODF_MINIMAX = 1, ODF_RGB = 2 } odf_dist;

/* Library version, (major << 16) | minor. */
int odf_version(void);

/* Message of the last failed call on this thread ("" if none).  The pointer
 * stays valid until the next failing call on the same thread. */
const char* odf_last_error(void);

/*
 * Forward filter, uint8 images (Section II; eqs. 1-3 with the pair term
 * chosen by `dist`).
 *   img   B x M x N x 3 uint8, read only.
 *   out   B x M x N x 3 uint8: out(b,r,c) is an exact copy of the selected
 *         window member.
 *   idx   B x M x N uint8 or NULL: the selected member index u in 0..n-1.
 *         Ties go to the lowest index.
 *   window any odd size from 3 to 15 (n = window^2 <= 225, so that the index
 *         fits a byte); kind ODF_BVDF / ODF_DDF; p in [0, 1] (DDF only,
 *         ignored by BVDF); dist ODF_EXACT / ODF_MINIMAX / ODF_RGB; q in
 *         {2, 3, 4} for ODF_MINIMAX (ignored otherwise).
 * Windows 3 to 9 run the tile and strip kernels (configs of the tuning
 * table); 11, 13 and 15 run a direct form with no configs: one workgroup per
 * 8 x 8 block of windows, every pair term of a window evaluated by the member
 * that needs it (the tile kernels' n aggregates per thread stop fitting the
 * registers past 9 x 9, 81 members).
 * Zero pixels take the direction (1,1,1) in the angle and chromaticity terms.
 * Errors: ODF_EINVAL for null img/out, sizes < 1, out overlapping img, or a
 * parameter out of range; ODF_EUNSUPPORTED for an even window or one outside
 * 3 to 15; ODF_EHIP if the launch fails.
 */
int odf_filter_u8(const uint8_t* img, int B, int M, int N, int window, int kind, float p,
                  int dist, int q, uint8_t* out, uint8_t* idx, void* stream);

/*
 * Forward filter, float32 images: same contract as odf_filter_u8 with
 * img/out as B x M x N x 3 float32.  ODF_MINIMAX and ODF_RGB need
 * non-negative inputs (the cosine lies in [0, 1], Section 2.1; chromaticity
 * sums are positive, eq. 7); ODF_EXACT takes values of either sign.
 * Domain: finite values with |x| <= 2^62.  The angle and chromaticity terms
 * scale each pixel by a power of two first and hold for any such value; the
 * L2 term of DDF squares raw channel differences in binary32, so larger
 * values can overflow it, and pixels that differ by less than 2^-63 in every
 * channel get their L2 distance from subnormal squares (fewer significant
 * bits).  Nothing checks the values on the device.
 */
int odf_filter_f32(const float* img, int B, int M, int N, int window, int kind, float p,
                   int dist, int q, float* out, uint8_t* idx, void* stream);

/*
 * Adaptive centre-weighted DDF, ACWDDF (Section III, Experiment 2: the
 * switching rule and the centre weights of eq. 9), uint8 images.  Per window,
 * with d the centre member (n-1)/2:
 *   - the DDF selection of eq. (3): the member minimising A_u * D_u;
 *   - for k = lambda, lambda+1, lambda+2 the centre-weighted DDF selection
 *     y_k: the member minimising (sum_v w_v(k) A(x_u,x_v)) *
 *     (sum_v w_v(k) L2(x_u,x_v)), w_d(k) = n - 2k + 2 and w_v(k) = 1 for
 *     v != d (the weights of eq. 9 applied to both sums of eq. 3);
 *   - S = sum_k A(y_k, x_d) * L2(y_k, x_d); the output is the DDF selection
 *     when S > T and the centre member otherwise.
 * A is the pair term of `dist` (exact angle, minimax of Table 1, or eq. 10
 * applied to the chromaticity distance), L2 eq. (1) with p = 2.  Ties in each
 * selection go to the lowest index.
 *   img, out, idx  as for odf_filter_u8 (idx = the output member: the DDF
 *          selection or (n-1)/2).
 *   lambda in [1, (n+1)/2 - 2] (so every level k lies in [1, (n+1)/2]); the
 *          paper's setting is lambda = 2, T = 10.8 (angles in radians, L2 in
 *          the units of the image values).
 *   T      any value but NaN (+inf keeps every centre; below 0 gives the DDF).
 * Any odd window from 3 to 15: 3 to 7 on the tile (and, to 5, strip)
 * kernels, 9 to 15 on the direct form of odf_filter_u8's large windows (no
 * configs).
 * Errors: as odf_filter_u8, plus ODF_EINVAL for lambda out of range or T NaN.
 */
int odf_acwddf_u8(const uint8_t* img, int B, int M, int N, int window, int dist, int q,
                  int lambda, float T, uint8_t* out, uint8_t* idx, void* stream);

/* ACWDDF on float32 images (same contract; ODF_MINIMAX and ODF_RGB need
 * non-negative inputs). */
int odf_acwddf_f32(const float* img, int B, int M, int N, int window, int dist, int q,
                   int lambda, float T, float* out, uint8_t* idx, void* stream);

/*
 * Centre-weighted filters at one smoothing level k (Section III, eq. 9), with
 * the centre member d = (n-1)/2 weighted w_d(k) = n - 2k + 2 and every other
 * member 1:
 *   ODF_CWVMF  CWVMF^k, eq. (9): the member minimising
 *              sum_v w_v(k) L2(x_u, x_v); `dist` and `q` are ignored;
 *   ODF_CWDDF  CWDDF^k: the same weights on both sums of eq. (3), the member
 *              minimising (sum_v w_v(k) A(x_u, x_v)) (sum_v w_v(k) L2(x_u, x_v)),
 *              A the pair term of `dist` as in odf_acwddf_u8.
 * k = d weighs every member 1 (CWVMF^d is the vector median, CWDDF^d the DDF
 * of eq. 3); k = 1 weighs the centre n, which keeps the centre's colour.
 *   level  k in [1, (n+1)/2].
 *   img, out, idx as for odf_filter_u8; ties go to the lowest index.
 * Runs on the ACWDDF sweep, with tile table entries of its own (kind
 * ODF_CWVMF or ODF_CWDDF in the tuning calls) for windows 3 to 7; windows 9 to
 * 15 (odd) run the direct form, which has no configs.
 * Errors: as odf_filter_u8, plus ODF_EINVAL for kind or level out of range.
 */
int odf_cw_filter_u8(const uint8_t* img, int B, int M, int N, int window, int kind, int dist, int q,
                     int level, uint8_t* out, uint8_t* idx, void* stream);
int odf_cw_filter_f32(const float* img, int B, int M, int N, int window, int kind, int dist, int q,
                      int level, float* out, uint8_t* idx, void* stream);

/*
 * Aggregates of every window (test and inspection hook, not the fast path).
 *   img    uint8 (is_u8 != 0) or float32 image as above.
 *   A      B x M x N x n float32: A[.., u] = sum_v theta(x_u, x_v), the pair
 *          term of `dist` (self pair included).
 *   D      B x M x N x n float32 or NULL: sum_v |x_u - x_v|_2 (DDF only;
 *          written as 0 for BVDF).
 *   Omega  B x M x N x n float32 or NULL: the objective the argmin uses
 *          (A for BVDF; A^(1-p) D^p for DDF).
 * Errors as for odf_filter_u8; windows 3 to 9 only (ODF_EUNSUPPORTED above).
 */
int odf_aggregates_f32(const void* img, int is_u8, int B, int M, int N, int window, int kind,
                       float p, int dist, int q, float* A, float* D, float* Omega, void* stream);

/*
 * Gradient of the hard filter (one-hot routing of the selection).
 *   idx  B x M x N uint8 from odf_filter_* (read only).
 *   dy   B x M x N x 3 float32 upstream gradient dL/dy.
 *   dx   B x M x N x 3 float32 output: dx(q) = sum of dy(c) over the windows c
 *        whose selected member is the pixel q (replicated border: a window
 *        selecting an out-of-image position selects its clamped source).  Each
 *        sum is formed in binary64 over c in raster order and rounded once.
 *        An index entry >= window^2 (not produced by the filter) routes
 *        nothing: its dy(c) reaches no pixel.
 * The forward selection is not touched.  Errors: ODF_EINVAL for null
 * pointers, sizes, or dx overlapping dy/idx; ODF_EUNSUPPORTED for an even
 * window or one outside 3 to 15.
 */
int odf_backward_hard_f32(const uint8_t* idx, const float* dy, int B, int M, int N, int window,
                          float* dx, void* stream);

/*
 * Softmin relaxation of the argmin (exact angle of eq. 2; kind/p as for the
 * filter): per window c, pi_u = exp(-(Omega_u - min_v Omega_v) / tau) / Z and
 * y(c) = sum_u pi_u x_u.  tau -> 0 tends to the hard selection where the
 * minimum is unique.
 *   x  B x M x N x 3 float32 (read only); y  B x M x N x 3 float32 output.
 * Any odd window from 3 to 15: 3 to 9 on LDS tiles, 11 to 15 on a direct form
 * (one thread per window, every pair term evaluated; far slower).
 * Errors: as odf_filter_f32, plus ODF_EINVAL for tau <= 0 or not finite.
 */
int odf_softmin_fwd_f32(const float* x, int B, int M, int N, int window, int kind, float p,
                        float tau, float* y, void* stream);

/* Workspace bytes odf_softmin_bwd_f32 needs for this shape (0 if invalid). */
size_t odf_softmin_bwd_workspace(int B, int M, int N, int window, int kind);

/*
 * Gradient of sum(dy * y) for the softmin relaxation, with respect to x:
 * through the weights pi (and so through Omega, the angle aggregates A and the
 * L2 aggregates D down to every pixel) and through the direct term pi_u.
 * Conventions where the derivative does not exist: the angle gradient is 0
 * for parallel pairs and zero pixels, the L2 gradient 0 for equal pixels,
 * dOmega/dA (dD) 0 where A (D) is 0 under a fractional power.
 *   dy         B x M x N x 3 float32 upstream gradient.
 *   dx         B x M x N x 3 float32 output.
 *   workspace  device scratch of at least odf_softmin_bwd_workspace() bytes,
 *              owned by the caller; its contents on entry are ignored.
 * Deterministic: the result does not depend on scheduling.
 */
int odf_softmin_bwd_f32(const float* x, const float* dy, int B, int M, int N, int window, int kind,
                        float p, float tau, float* dx, void* workspace, size_t workspace_bytes,
                        void* stream);

/*
 * odf_softmin_bwd_f32 without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments (minus the workspace),
 * contract, result (bit for bit) and errors as odf_softmin_bwd_f32; the
 * workspace is a static device array of the library of 128 MiB (2^27 bytes),
 * one copy per GPU, held from the library's load until the process ends.
 * Shapes whose odf_softmin_bwd_workspace() exceeds 2^27 bytes are rejected with
 * ODF_EINVAL (16 x 512 x 512 at 5x5 needs 77 MiB and fits).  The call allocates
 * nothing and does not synchronise; the first call on a device looks up the
 * array's address there (hipGetSymbolAddress), which needs that device current
 * and `stream` to belong to it.  Every call on one GPU uses the same array:
 * calls that overlap in time on one GPU (concurrent streams, or threads)
 * race and must be serialised by the caller; calls on one stream are ordered.
 */
int odf_softmin_bwd_f32_noalloc(const float* x, const float* dy, int B, int M, int N, int window,
                                int kind, float p, float tau, float* dx, void* stream);

/*
 * binary64 twins of the softmin relaxation and its gradient, for gradient
 * checks by finite differences in binary64 (the float32 entry points above are
 * the fast path).  Same definitions, conventions and errors as
 * odf_softmin_fwd_f32 / odf_softmin_bwd_f32, with x, y, dy, dx binary64
 * (B x M x N x 3) and p, tau binary64; every pair term, aggregate, weight and
 * gradient is formed in binary64 directly from its definition, one window per
 * thread (no tiles, no reuse of pair terms), so these run far slower than the
 * float32 path.  The backward first writes the gradient of every member of
 * every window to the workspace (n x 3 binary64 per pixel, 8-byte aligned,
 * owned by the caller, contents on entry ignored), then sums, for every pixel,
 * those of the members that are that pixel (windows in raster order, members
 * in index order): deterministic.  Windows 3, 5, 7 and 9.
 */
int odf_softmin_fwd_f64(const double* x, int B, int M, int N, int window, int kind, double p,
                        double tau, double* y, void* stream);

/* Workspace bytes odf_softmin_bwd_f64 needs (B M N n 3 8; 0 if invalid). */
size_t odf_softmin_bwd_f64_workspace(int B, int M, int N, int window);

int odf_softmin_bwd_f64(const double* x, const double* dy, int B, int M, int N, int window, int kind,
                        double p, double tau, double* dx, void* workspace, size_t workspace_bytes,
                        void* stream);

/* ---------------------------------------------------------------- batches
 * Many uint8 images of different sizes, windows and variants in one launch.
 * A job is one image with its own parameters (same meaning as the arguments
 * of odf_filter_u8; idx may be NULL; windows 3, 5, 7 and 9, kinds ODF_BVDF and
 * ODF_DDF).  Results are bitwise equal to those of odf_filter_u8 on each
 * image. */
typedef struct {
    const uint8_t* img; /* M x N x 3 uint8 */
    uint8_t* out;       /* M x N x 3 uint8 */
    uint8_t* idx;       /* M x N uint8 or NULL */
    int M, N;
    int window, kind, dist, q;
    float p;
} odf_job;

typedef struct odf_plan odf_plan; /* opaque, owned by the library */

/* Validate the jobs, cut them into tiles (or strips) and upload the work lists
 * (one per group of window and kind, holding the items of every pair term,
 * heavier items first); each group runs on the config (tile shape or strip
 * height) the batch tuning table holds for it when the plan is made
 * (odf_batch_tune_get, odf_autotune_batch).  Allocates device memory and synchronises; the job
 * buffers must stay valid while the plan is launched.  On success *plan
 * receives a plan to pass to odf_batch_launch and finally to
 * odf_plan_destroy.  Errors: ODF_EINVAL / ODF_EUNSUPPORTED for a bad job
 * (nothing is allocated), ODF_ENOMEM, ODF_EHIP. */
int odf_batch_plan(const odf_job* jobs, int njobs, odf_plan** plan, void* stream);

/* odf_batch_plan with a launch form.  ODF_BATCH_DIRECT (one workgroup per tile
 * of the work list, dispatched in list order) is odf_batch_plan.
 * ODF_BATCH_PERSISTENT (persistent workgroups taking tiles from an atomic
 * counter) is retired and returns ODF_EUNSUPPORTED: measured on MI355X it ran
 * at 0.6 of the direct form (its loop cost registers), and the direct form
 * already runs the groups at the kernels' own steady-state rate. */
enum { ODF_BATCH_PERSISTENT = 0, ODF_BATCH_DIRECT = 1 };
int odf_batch_plan_ex(const odf_job* jobs, int njobs, int flags, odf_plan** plan, void* stream);

/* Enqueue the plan on `stream`: one kernel per non-empty group over its work
 * list; a group kernel runs the tiles of all three pair terms of its window
 * and kind.  Groups after the first run on the plan's own auxiliary streams,
 * forked from and joined back to `stream` with events, so they overlap;
 * everything is ordered after prior work on `stream` and before later work on
 * it.  Allocates nothing and does not synchronise, so it may be captured in a
 * hipGraph and replayed.  Launches of one plan must not overlap in time (they
 * share the plan's streams). */
int odf_batch_launch(const odf_plan* plan, void* stream);

/* Plan summary: job count, total pixels, and per class of window, kind and
 * pair term, class = (((window - 3) / 2) * 2 + kind) * 3 + dist (arrays of 24, each
 * nullable): its tiles, and the workgroups launched for them (one per tile). */
int odf_plan_info(const odf_plan* plan, int* njobs, long long* npix, int* ntiles, int* grids);

/* The config each group of the plan runs on (a tile shape, odf_tile_config
 * number, or a strip config), group = ((window - 3) / 2) * 2 + kind, configs[8].
 * ODF_EINVAL for NULL. */
int odf_plan_configs(const odf_plan* plan, int* configs);

/* Free a plan (after its last launch has completed). */
int odf_plan_destroy(odf_plan* plan);

/* ---------------------------------------------------------------- noise and quality
 * The correlated impulsive noise model of eq. (8) and the MAE / PSNR measures
 * of Section III, for effectiveness checks on synthetic clean/noisy pairs. */

/*
 * noisy = clean corrupted by eq. (8): with probability phi a pixel is
 * corrupted, then only its red, green or blue channel (probabilities phi_r,
 * phi_g, phi_b) or all three (the rest) take the values of a random vector r
 * uniform in {0..255}^3; otherwise it is copied.
 * Random numbers: pixel i = (b*M + row)*N + col draws one Philox4x32-10 block
 * (Salmon et al., SC 2011) with counter (i mod 2^32, i div 2^32, 0, 0) and key
 * (seed mod 2^32, seed div 2^32): word 0 < floor(phi 2^32) corrupts; word 1
 * against floor(phi_r 2^32), floor((phi_r + phi_g) 2^32),
 * floor((phi_r + phi_g + phi_b) 2^32) picks red only, green only, blue only,
 * else all three; bytes 0, 1, 2 of word 2 are r.  Results depend only on
 * (seed, i), not on the launch.
 *   clean, noisy  B x M x N x 3 uint8; noisy may equal clean (in place) but
 *                 must not partially overlap it.
 * Errors: ODF_EINVAL for null pointers, sizes (B*M*N >= 2^40), phi outside
 * [0, 1], a negative channel probability or phi_r + phi_g + phi_b > 1.
 */
int odf_noise_eq8_u8(const uint8_t* clean, uint8_t* noisy, int B, int M, int N, double phi,
                     double phi_r, double phi_g, double phi_b, uint64_t seed, void* stream);

/* Workspace bytes odf_quality_u8 needs for B images (0 if B < 1). */
size_t odf_quality_workspace(int B);

/*
 * Per image b of B: MAE = sum |y - ref| / (3MN) and
 * PSNR = 10 log10(255^2 / MSE), MSE = sum (y - ref)^2 / (3MN), over the three
 * channels of every pixel (Section III; PSNR = +inf for identical images).
 * The sums are exact 64-bit integers, so the results do not depend on
 * scheduling.
 *   y, ref     B x M x N x 3 uint8 (read only).
 *   mae, psnr  B float64 each, device memory.
 *   workspace  device scratch of odf_quality_workspace(B) bytes, 8-byte
 *              aligned, owned by the caller; contents on entry ignored.
 * Errors: ODF_EINVAL for null pointers, sizes (B > 65535 or B*M*N >= 2^40)
 * or a short / misaligned workspace.
 */
int odf_quality_u8(const uint8_t* y, const uint8_t* ref, int B, int M, int N, double* mae,
                   double* psnr, void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------- tuning
 * The forward kernels run one thread per pixel of an extended tile
 * (output tile plus halo).  Configs 0..3 are tile shapes (one workgroup per
 * output tile); configs ODF_STRIP_CONFIG (4) and ODF_SHORT_STRIP_CONFIG (5) are
 * the strip form, offered for ODF_BVDF and ODF_DDF at 3x3, 5x5 and 7x7, for
 * ODF_BVDF at 9x9 on uint8 and for the centre-weighted kinds at 3x3 to 7x7
 * (the batch offers them for all its groups): one
 * workgroup per strip of 32 - 2h output columns and 8 * 16 - 2h (config 4) or
 * 3 * 16 - 2h (config 5, for images too small to fill the GPU with long
 * strips) output rows, walking down it in bands of 32 x 16 member pixels and
 * keeping the pair terms and argmin keys that consecutive bands share in LDS,
 * so that the rows of the halo between bands are not evaluated twice (results
 * bitwise equal to the tile shapes).  odf_tile_config
 * gives the extended width and height of a tile shape, or of one band of the
 * strip form.  The process-wide table picks a config per (window, kind,
 * dist, input type), kind any odf_kind (windows 3 to 9; 3, 5 and 7 for
 * ODF_ACWDDF, ODF_CWVMF and ODF_CWDDF; ODF_CWVMF has no angular term and keeps one entry
 * for every dist); the default is shape 2 (32 x 16) for every class (the 5x5
 * centre-weighted kinds and 7x7 offer only the 512-thread shapes 2 and 3 and,
 * where the strip form covers them, configs 4 and 5; 9x9 only shape 2 and the
 * strips).  The table is initialised once per process and each entry is
 * read and written atomically. */
#define ODF_NUM_TILE_CONFIGS 6
#define ODF_STRIP_CONFIG 4
#define ODF_SHORT_STRIP_CONFIG 5
int odf_tile_config(int config, int* ext_w, int* ext_h);
int odf_tune_get(int window, int kind, int dist, int is_u8);                  /* config or < 0 */
int odf_tune_set(int window, int kind, int dist, int is_u8, int config);      /* ODF_EINVAL if invalid */

/* Time every config the class offers on a seeded M x N tuning image (a smooth
 * field with 15 % impulsive noise; reps launches each, HIP events on
 * `stream`), set the fastest in the table, store the per-config milliseconds
 * in times_ms[ODF_NUM_TILE_CONFIGS] (-1 for configs not offered; nullable)
 * and append one JSON line to cache_path (nullable).  Allocates and frees
 * device memory and synchronises `stream`.  Errors: ODF_EINVAL (class or
 * sizes out of range, M*N >= 2^28), ODF_ENOMEM (host or device allocation
 * failed), ODF_EHIP. */
int odf_autotune(int window, int kind, int dist, int is_u8, int M, int N, int reps,
                 const char* cache_path, float* times_ms, void* stream);

/* The batch tuning table: the config (0..3 a tile shape, ODF_STRIP_CONFIG or
 * ODF_SHORT_STRIP_CONFIG the strip form) of the batch group of
 * `window` (3, 5, 7, 9) and `kind` (ODF_BVDF, ODF_DDF); 32 x 32 for 3x3 DDF and
 * 32 x 16 otherwise until tuned.  get returns the config or ODF_EINVAL; set
 * returns ODF_OK, or ODF_EINVAL for a config the group does not offer (7x7:
 * the 512-thread shapes 2 and 3 and the strips; 9x9: shape 2 and, for
 * ODF_BVDF, the strips; as odf_tune_set for uint8).  Plans read
 * the table when they are made. */
int odf_batch_tune_get(int window, int kind);
int odf_batch_tune_set(int window, int kind, int config);

/* Time the ODF_NUM_TILE_CONFIGS configs of one batch group on a seeded mixed
 * work list (six tuning images from 64 x 64 to 1920 x 1080, each with the
 * three pair terms: 18 jobs; reps launches per config, HIP events on
 * `stream`), set the fastest in the batch table, store the per-config
 * milliseconds in times_ms[ODF_NUM_TILE_CONFIGS] (-1 for a config
 * the group does not offer; nullable) and append one JSON line to cache_path (nullable).  Allocates
 * and frees device memory and synchronises `stream`.  Errors: ODF_EINVAL,
 * ODF_ENOMEM, ODF_EHIP. */
int odf_autotune_batch(int window, int kind, int reps, const char* cache_path, float* times_ms,
                       void* stream);

/* The same on the caller's own jobs (validated as for odf_batch_plan): for each
 * batch group that holds jobs, its configs are timed on the group's jobs (reps
 * launches each; the jobs' outputs are written) and the fastest is set in the
 * batch table and appended to cache_path (nullable);
 * times_ms[ODF_NUM_TILE_CONFIGS * group + config] (nullable, 8 *
 * ODF_NUM_TILE_CONFIGS floats) receives the milliseconds, -1 for groups
 * without jobs and for configs a group does not offer.  A plan made afterwards for the same jobs runs
 * on the shapes tuned for them.  Errors: as odf_batch_plan. */
int odf_autotune_batch_jobs(const odf_job* jobs, int njobs, int reps, const char* cache_path,
                            float* times_ms, void* stream);

/* Apply the entries of a cache written by odf_autotune or odf_autotune_batch
 * whose architecture matches the current device; returns the number applied
 * or ODF_EINVAL. */
int odf_tune_load(const char* cache_path);

#ifdef __cplusplus
}
#endif

#endif /* ODF_H */
