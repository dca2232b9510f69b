// pair_terms.h -- device-side pixel preparation and pair terms of the
// directional filters (Section II and Sections 2.1-2.2 of Celebi,
// arXiv:1009.0958), in binary32 on the VALU of gfx950.
//
// Each prepared pixel is two float4 values:
//   dir = (d.x, d.y, d.z, aux1)   d: direction (the pixel, or (1,1,1) for 0)
//   raw = (x.x, x.y, x.z, aux2)   x: the raw pixel
//   EXACT:   aux1 = |x|^2, or -3 for x = 0 (|d|^2 = 3 for d = (1,1,1); the sign
//            marks the zero pixel), aux2 = |d| / |x| (a power of two; 0 for x = 0)
//   MINIMAX: aux1 = |d|^2, aux2 = 1/|d|
//   RGB:     aux1 = d.x + d.y + d.z, aux2 = 1/aux1
//
// Every pair term is symmetric bit for bit (term(a,b) == term(b,a)) and
// returns for a pair of equal vectors exactly the value it returns for the
// self pair, so equal colours in a window get bitwise-equal aggregates.
// Cross-product and chromaticity numerators are differences of two rounded
// products (no fused multiply-add), which keeps swapped arguments exact
// negations; for uint8 inputs they are exact integers, formed with one fused
// multiply-add.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "atan_poly.h"

namespace odf {

// kACW: the adaptive centre-weighted DDF (Section III, Experiment 2), whose
// pair terms are the DDF's.
enum Kind { kBVDF = 0, kDDF = 1, kACW = 2 };
enum Dist { kExact = 0, kMinimax = 1, kRgb = 2 };

// eq. (10): A ~= 1.436437 B + 0.027664
constexpr float kEq10Alpha = 1.436437f;
constexpr float kEq10Beta = 0.027664f;

constexpr float kHalfPi = 1.57079632679489661923f;
constexpr float kPi = 3.14159265358979323846f;

// a*b - c*d with both products rounded separately.
__device__ __forceinline__ float diff_of_products(float a, float b, float c, float d) {
#pragma clang fp contract(off)
    return a * b - c * d;
}

// a*b - c*d of a cross product or chromaticity numerator.  EXACT_INT: uint8
// pixels, integer operands whose products (at most 255 * 765) and their
// difference are exact in binary32, so one fused multiply-add yields the same
// exact, hence symmetric, value.
template <bool EXACT_INT>
__device__ __forceinline__ float cross_diff(float a, float b, float c, float d) {
    if constexpr (EXACT_INT) return fmaf(a, b, -(c * d));
    else return diff_of_products(a, b, c, d);
}

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float sqrt_raw(float x) { return __builtin_amdgcn_sqrtf(x); }

// Table 1 coefficients, zero-padded to degree 4 (Horner with leading zeros
// reproduces the degree-q evaluation exactly).
struct MinimaxCoef {
    float asin_c[5];
    float acos_c[5];
};

__device__ __forceinline__ float horner4(const float* c, float t) {
    float acc = c[4];
    acc = fmaf(acc, t, c[3]);
    acc = fmaf(acc, t, c[2]);
    acc = fmaf(acc, t, c[1]);
    acc = fmaf(acc, t, c[0]);
    return acc;
}

// Prepare one pixel.  For float inputs the direction is scaled by a power of
// two (exact; angles and chromaticities are scale-free) so that its largest
// magnitude lies in [1, 2), which keeps every product below in range.
template <int DIST, bool U8>
__device__ __forceinline__ void prepare_pixel(float x0, float x1, float x2, float4& dir,
                                              float4& raw) {
    float d0 = x0, d1 = x1, d2 = x2;
    const bool zero = (x0 == 0.0f) & (x1 == 0.0f) & (x2 == 0.0f);
    int e = 0;
    if (!U8) {
        const float m = fmaxf(fabsf(x0), fmaxf(fabsf(x1), fabsf(x2)));
        e = zero ? 0 : ilogbf(m);
        d0 = ldexpf(x0, -e);
        d1 = ldexpf(x1, -e);
        d2 = ldexpf(x2, -e);
    }
    if (zero) d0 = d1 = d2 = 1.0f;
    float aux1 = 0.0f, aux2 = 0.0f;
    if (DIST == kExact) {
        // |x|^2 of the raw value (exact for uint8), and d = 2^-e x: the
        // derivative of the direction (0 for the zero pixel, whose direction
        // is a constant), used by the angle gradient
        aux1 = zero ? -3.0f : fmaf(x0, x0, fmaf(x1, x1, x2 * x2));
        aux2 = zero ? 0.0f : ldexpf(1.0f, -e);
    } else if (DIST == kMinimax) {
        aux1 = fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
        aux2 = 1.0f / sqrtf(aux1);
    } else if (DIST == kRgb) {
        aux1 = (d0 + d1) + d2;
        aux2 = 1.0f / aux1;
    }
    dir = make_float4(d0, d1, d2, aux1);
    raw = make_float4(x0, x1, x2, aux2);
}

// Exact angle of eq. (2), evaluated as atan2(|a x b|, a.b):
// with P = |a x b|^2 and Q = (a.b)^2, r = sqrt(min(P,Q)/max(P,Q)) =
// min(P,Q) / sqrt(P Q) lies in [0, 1] and the angle is atan(r) or
// pi/2 - atan(r); one reciprocal square root per pair.
// |a x b|^2.  uint8 (U8): Lagrange's identity |a|^2 |b|^2 - (a.b)^2 in
// binary64, exact (every operand an integer below 2^53), from the squared
// direction norms na, nb and the dot product; otherwise the sum of the squared
// cross components.
template <bool U8>
__device__ __forceinline__ float cross_norm2(const float4& a, const float4& b, float na, float nb,
                                             float dot) {
    if constexpr (U8) {
        const double d = (double)dot;
        return (float)fma(-d, d, (double)na * (double)nb);
    } else {
        float c0 = cross_diff<U8>(a.y, b.z, a.z, b.y);
        float c1 = cross_diff<U8>(a.z, b.x, a.x, b.z);
        float c2 = cross_diff<U8>(a.x, b.y, a.y, b.x);
        return fmaf(c0, c0, fmaf(c1, c1, c2 * c2));
    }
}

template <bool U8>
__device__ __forceinline__ float angle_exact_dot(const float4& a, const float4& b, float& dot) {
    constexpr bool SIGNED = !U8;  // float inputs may be negative
    dot = fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z));
    // |d|^2 = |aux1| (the zero pixel's -3 stands for |(1,1,1)|^2)
    float P = cross_norm2<U8>(a, b, fabsf(a.w), fabsf(b.w), dot);
    float Q = dot * dot;
    float m = fminf(P, Q);
    float r = m * rsq(fmaxf(P * Q, 1.17549435e-38f));
    float t = r * r;
    float acc = kAtanPoly[ODF_ATAN_DEG];
#pragma unroll
    for (int k = ODF_ATAN_DEG - 1; k >= 0; --k) acc = fmaf(acc, t, kAtanPoly[k]);
    float at = r * acc;
    float th = (P > Q) ? (kHalfPi - at) : at;
    if (SIGNED) th = (dot < 0.0f) ? (kPi - th) : th;
    return th;
}

template <bool U8>
__device__ __forceinline__ float angle_exact(const float4& a, const float4& b) {
    float dot;
    return angle_exact_dot<U8>(a, b, dot);
}

// Method 1 (Section 2.1): ACOS row of Table 1 in z for z < 1/2, ASIN row in
// tau = sqrt(1 - z) for z >= 1/2 (eqs. 5-6), clamped at 0.  The branch is the
// exact predicate 4 (a.b)^2 < |a|^2 |b|^2 (binary64 products of binary32
// values are exact).  The binary32 cosine z = a.b / (|a| |b|) is within a few
// ulp of the true one (a.b is exact or nearly so for non-negative inputs, the
// reciprocal norms are correctly rounded), so outside |z - 1/2| <= 2^-20 its
// own comparison gives the same answer and the binary64 test is skipped.
// 1 - z = |a x b|^2 / (|a|^2 |b|^2 (1 + z)) avoids the cancellation of 1 - z
// next to z = 1.
template <bool U8>
__device__ __forceinline__ float angle_minimax(const float4& a, const float4& ra, const float4& b,
                                               const float4& rb, const MinimaxCoef& cf) {
    float dot = fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z));
    float z = dot * (ra.w * rb.w);
    bool acos_branch = z < 0.5f;
    const bool near = fabsf(z - 0.5f) <= 0x1p-20f;
    if (__builtin_amdgcn_ballot_w64(near)) {  // uniform branch, almost never taken
        asm volatile("");                     // keeps the exact test out of the common path
        if (near) acos_branch = 4.0 * (double)dot * (double)dot < (double)a.w * (double)b.w;
    }
    float P = cross_norm2<U8>(a, b, a.w, b.w, dot);
    float X = (a.w * b.w) * (1.0f + z);
    float tau = P * rsq(fmaxf(P * X, 1.17549435e-38f));
    // the clamp at 0 matters for the ASIN row only (q = 3 dips below 0 next to
    // tau = 0); every ACOS row stays above 1 on [-1, 1/2]
    return acos_branch ? horner4(cf.acos_c, z) : fmaxf(horner4(cf.asin_c, tau), 0.0f);
}

// Method 2 (Section 2.2, eq. 7): L2 distance of chromaticities
// |a / sum a - b / sum b| = |a sum b - b sum a| / (sum a sum b).
template <int KIND, bool U8>
__device__ __forceinline__ float chroma_term(const float4& a, const float4& ra, const float4& b,
                                             const float4& rb) {
    float n0 = cross_diff<U8>(a.x, b.w, b.x, a.w);
    float n1 = cross_diff<U8>(a.y, b.w, b.y, a.w);
    float n2 = cross_diff<U8>(a.z, b.w, b.z, a.w);
    float Nn = fmaf(n0, n0, fmaf(n1, n1, n2 * n2));
    float B = sqrt_raw(Nn) * (ra.w * rb.w);
    if (KIND != kBVDF) B = fmaf(kEq10Alpha, B, kEq10Beta);  // eq. (10), Experiment 2
    return B;
}

// Angular pair term of the chosen variant.
template <int KIND, int DIST, bool U8>
__device__ __forceinline__ float pair_term(const float4& a, const float4& ra, const float4& b,
                                           const float4& rb, const MinimaxCoef& cf) {
    if (DIST == kExact) return angle_exact<U8>(a, b);
    if (DIST == kMinimax) return angle_minimax<U8>(a, ra, b, rb, cf);
    return chroma_term<KIND, U8>(a, ra, b, rb);
}

// eq. (1) with the L2 norm (Section III), on raw values.
__device__ __forceinline__ float l2_term(const float4& ra, const float4& rb) {
    float e0 = ra.x - rb.x, e1 = ra.y - rb.y, e2 = ra.z - rb.z;
    return sqrt_raw(fmaf(e0, e0, fmaf(e1, e1, e2 * e2)));
}

// The angular pair term of member a (dir a, raw ra) with neighbour q of the
// LDS tile, and their L2 distance of eq. (1) in l2.  For uint8 exact angles the
// squared distance reuses the dot product of the angle:
// |x_a - x_b|^2 = |x_a|^2 + |x_b|^2 - 2 x_a.x_b, every term an integer exact in
// binary32, with |x|^2 in dir.w.  A zero pixel (direction (1,1,1), value 0,
// dir.w = -3) has a zero raw dot product and |x|^2 = 0; the lanes with one take
// max(dir.w, 0) summed over the pair in a branch the wave enters only when some
// lane needs it.
template <int KIND, int DIST, bool U8>
__device__ __forceinline__ float pair_and_l2(const float4& a, const float4& ra,
                                             const float4* __restrict__ s_dir,
                                             const float4* __restrict__ s_raw, int q,
                                             const MinimaxCoef& cf, float& l2) {
    const float4 b = s_dir[q];
    if constexpr (DIST == kExact && U8) {
        float dot;
        const float th = angle_exact_dot<U8>(a, b, dot);
        float l2sq = fmaf(-2.0f, dot, a.w + b.w);
        const bool zero = (__float_as_int(a.w) | __float_as_int(b.w)) < 0;  // a sign set
        if (__builtin_amdgcn_ballot_w64(zero)) {
            asm volatile("");  // keeps the fix-up out of the common path
            if (zero) l2sq = fmaxf(a.w, 0.0f) + fmaxf(b.w, 0.0f);
        }
        l2 = sqrt_raw(l2sq);
        return th;
    } else {
        const float4 rb = s_raw[q];
        l2 = l2_term(ra, rb);
        return pair_term<KIND, DIST, U8>(a, ra, b, rb, cf);
    }
}

// Total order on floats (no NaN) as unsigned keys.
__device__ __forceinline__ uint32_t order_key(float v) {
    uint32_t bits = __float_as_uint(v + 0.0f);  // -0 -> +0
    return (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);
}

}  // namespace odf
