// pair_terms.h -- device-side pixel preparation and pair terms of the
// directional filters (Section II and Sections 2.1-2.2 of Celebi,
// arXiv:1009.0958), in binary32 on the VALU of gfx950.
//
// A prepared float pixel is two float4 values:
//   dir = (d.x, d.y, d.z, aux1)   d: direction (the pixel scaled by a power of
//                                    two, or (1,1,1) for 0)
//   raw = (x.x, x.y, x.z, aux2)   x: the raw pixel
//   EXACT:   aux1 = |x|^2, or -3 for x = 0, aux2 = |d| / |x| (0 for x = 0)
//   MINIMAX: aux1 = |d|^2, aux2 = 1/|d|
//   RGB:     aux1 = d.x + d.y + d.z, aux2 = 1/aux1
// A prepared uint8 pixel is dir alone, with d = x (exact integers) or (1,1,1)
// for the zero pixel, plus aux2 for MINIMAX and RGB: aux1 = |x|^2 (EXACT,
// MINIMAX) or the channel sum (RGB), and -3 for the zero pixel (|d|^2 and the
// sum of (1,1,1) are 3; the sign marks the zero pixel).  The raw value is
// dir.xyz, or 0 where aux1 < 0.
//
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "atan_poly.h"

namespace odf {

// kACW: the adaptive centre-weighted DDF (Section III, Experiment 2), whose
// pair terms are the DDF's.
enum Kind { kBVDF = 0, kDDF = 1, kACW = 2, kCW = 3, kCWV = 4 };
// kCW: CWDDF^k, one centre-weighted DDF at one level, on the ACWDDF sweep
// (which forms every member's terms with the window centre); kCWV: CWVMF^k,
// the same with the L2 sweep alone (eq. 9 has no angle).
constexpr bool centre_weighted(int kind) { return kind == kACW || kind == kCW || kind == kCWV; }
enum Dist { kExact = 0, kMinimax = 1, kRgb = 2 };

// eq. (10): A ~= 1.436437 B + 0.027664
constexpr float kEq10Alpha = 1.436437f;
constexpr float kEq10Beta = 0.027664f;

constexpr float kHalfPi = 1.57079632679489661923f;
constexpr float kPi = 3.14159265358979323846f;

// c as a wave-uniform value in a scalar register, opaque to constant folding.
// A multiply-add then takes it as its scalar operand; left as a literal, the
// compiler tends to copy polynomial coefficients into vector registers, one
// VALU move each.
__device__ __forceinline__ float scalar_const(float c) {
    int z;
    asm("s_mov_b32 %0, 0" : "=s"(z));
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(c) | z));
}

// The atan polynomial's coefficients in scalar registers, formed once by the
// caller of a pair-term loop.
struct AtanCoef {
    float c[ODF_ATAN_DEG + 1];
};

__device__ __forceinline__ AtanCoef atan_coef() {
    AtanCoef a;
#pragma unroll
    for (int k = 0; k <= ODF_ATAN_DEG; ++k) a.c[k] = kAtanPoly[k];
    // all but c0 (1, an inline constant) and the second-highest, which the
    // first Horner step takes as its literal (c_deg t + c_deg-1 is then one
    // multiply-add with a scalar and a literal operand)
#pragma unroll
    for (int k = 1; k <= ODF_ATAN_DEG; ++k)
        if (k != ODF_ATAN_DEG - 1) a.c[k] = scalar_const(kAtanPoly[k]);
    return a;
}

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

// 1/sqrt(x) for a product x = u v that is 0 only when a factor u is 0, used as
// u * rsq_pos(x): the result must be finite at x = 0.  uint8 inputs (INT): x
// is 0 or at least 1, so rsq(x) lies in (0, 1] or is +inf at 0, and clamping
// to [0, 1] (the instruction's clamp modifier, free) maps +inf to 1;
// otherwise x is raised to the smallest normal number first.
template <bool INT>
__device__ __forceinline__ float rsq_pos(float x) {
    if constexpr (INT) return __builtin_amdgcn_fmed3f(rsq(x), 0.0f, 1.0f);
    else return rsq(fmaxf(x, 1.17549435e-38f));
}
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
// magnitude lies in [1, 2), which keeps every product below in range.  raw.w
// is aux2 in both layouts.  CANON (uint8 only): the direction is the canonical
// integer direction of canon.h, given as cd0..cd2, and aux1 is its own squared
// norm or channel sum (the kinds that use it have no L2 term, and the output
// is copied from the image).
template <int DIST, bool U8, bool CANON = false>
__device__ __forceinline__ void prepare_pixel(float x0, float x1, float x2, float4& dir,
                                              float4& raw, float cd0 = 0.0f, float cd1 = 0.0f,
                                              float cd2 = 0.0f) {
    static_assert(U8 || !CANON, "canonical directions are for uint8 pixels");
    float d0 = x0, d1 = x1, d2 = x2;
    const bool zero = (x0 == 0.0f) & (x1 == 0.0f) & (x2 == 0.0f);
    if (CANON) {
        d0 = cd0;
        d1 = cd1;
        d2 = cd2;
    }
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
        // |x|^2 of the raw value (exact for uint8; of the canonical direction
        // with CANON), and d = 2^-e x: the derivative of the direction (0 for
        // the zero pixel, whose direction is a constant), used by the angle
        // gradient
        const float s0 = CANON ? d0 : x0, s1 = CANON ? d1 : x1, s2 = CANON ? d2 : x2;
        aux1 = zero ? -3.0f : fmaf(s0, s0, fmaf(s1, s1, s2 * s2));
        aux2 = zero ? 0.0f : ldexpf(1.0f, -e);
    } else if (DIST == kMinimax) {
        // n2 >= 1 (uint8 integers, or float directions scaled into [1, 2)):
        // the hardware reciprocal square root (about 1 ulp) needs no range fix-up
        const float n2 = fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
        aux1 = (U8 && zero) ? -3.0f : n2;
        aux2 = __builtin_amdgcn_rsqf(n2);
    } else if (DIST == kRgb) {
        const float sum = (d0 + d1) + d2;
        aux1 = (U8 && zero) ? -3.0f : sum;
        aux2 = __builtin_amdgcn_rcpf(sum);  // about 1 ulp
    }
    dir = make_float4(d0, d1, d2, aux1);
    raw = make_float4(x0, x1, x2, aux2);
}

// aux1 of a prepared pixel as a norm or sum (uint8: without the zero mark).
template <bool U8>
__device__ __forceinline__ float aux_mag(float w) {
    return U8 ? fabsf(w) : w;
}

// Exact angle of eq. (2), evaluated as atan2(|a x b|, a.b):
// with P = |a x b|^2 and Q = (a.b)^2, r = sqrt(min(P,Q)/max(P,Q)) =
// min(P,Q) / sqrt(P Q) lies in [0, 1] and the angle is atan(r) or
// pi/2 - atan(r); one reciprocal square root per pair.
// |a x b|^2.  uint8 (U8): Lagrange's identity |a|^2 |b|^2 - (a.b)^2 in
// binary64, exact (every operand an integer below 2^53), from the squared
// direction norms na, nb and the dot product.  Float directions: the cross
// product in binary64, where the products of binary32 components are exact,
// so each component is the exact difference rounded once (a multiply-add of
// one exact product and the other gives the same value) and swapping a and b
// negates it exactly; its squared norm is rounded to binary32 once.  In
// binary32 the components of a nearly parallel pair would cancel to
// |a| |b| sin(theta) with an absolute error of about 2^-24 |a| |b|, a
// relative error of 2^-24 / theta in the angle.
template <bool U8>
__device__ __forceinline__ float cross_norm2(const float4& a, const float4& b, float na, float nb,
                                             float dot) {
    if constexpr (U8) {
        const double d = (double)dot;
        return (float)fma(-d, d, (double)na * (double)nb);
    } else {
        const double a0 = a.x, a1 = a.y, a2 = a.z, b0 = b.x, b1 = b.y, b2 = b.z;
        const double c0 = fma(a1, b2, -(a2 * b1));
        const double c1 = fma(a2, b0, -(a0 * b2));
        const double c2 = fma(a0, b1, -(a1 * b0));
        return (float)fma(c0, c0, fma(c1, c1, c2 * c2));
    }
}

template <bool U8>
__device__ __forceinline__ float angle_exact_from_dot(const float4& a, const float4& b, float dot,
                                                      const AtanCoef& ac) {
    constexpr bool SIGNED = !U8;  // float inputs may be negative
    // |d|^2 = |aux1| (the zero pixel's -3 stands for |(1,1,1)|^2)
    float P = cross_norm2<U8>(a, b, fabsf(a.w), fabsf(b.w), dot);
    float Q = dot * dot;
    float m = fminf(P, Q);
    float r = m * rsq_pos<U8>(P * Q);
    float t = r * r;
    float acc = ac.c[ODF_ATAN_DEG];
#pragma unroll
    for (int k = ODF_ATAN_DEG - 1; k >= 0; --k) acc = fmaf(acc, t, ac.c[k]);
    float at = r * acc;
    float th = (P > Q) ? (kHalfPi - at) : at;
    if (SIGNED) th = (dot < 0.0f) ? (kPi - th) : th;
    return th;
}

__device__ __forceinline__ float dot3(const float4& a, const float4& b) {
    return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z));
}

template <bool U8>
__device__ __forceinline__ float angle_exact(const float4& a, const float4& b, const AtanCoef& ac) {
    return angle_exact_from_dot<U8>(a, b, dot3(a, b), ac);
}

// Method 1 (Section 2.1): ACOS row of Table 1 in z for z < 1/2, ASIN row in
// tau = sqrt(1 - z) for z >= 1/2 (eqs. 5-6), clamped at 0.  The branch is the
// exact predicate 4 (a.b)^2 < |a|^2 |b|^2 (binary64 products of binary32
// values are exact).  The binary32 cosine z = a.b / (|a| |b|) is within a few
// ulp of the true one (a.b is exact or nearly so for non-negative inputs, the
// reciprocal norms are within about an ulp), so outside |z - 1/2| <= 2^-20 its
// own comparison gives the same answer and the binary64 test is skipped.
// 1 - z = |a x b|^2 / (|a|^2 |b|^2 (1 + z)) avoids the cancellation of 1 - z
// next to z = 1.
template <bool U8>
__device__ __forceinline__ float angle_minimax_from_dot(const float4& a, float ia, const float4& b,
                                                        float ib, float dot,
                                                        const MinimaxCoef& cf) {
    const float na = aux_mag<U8>(a.w), nb = aux_mag<U8>(b.w);
    float z = dot * (ia * ib);
    bool acos_branch = z < 0.5f;
    const bool near = fabsf(z - 0.5f) <= 0x1p-20f;
    if (__builtin_amdgcn_ballot_w64(near)) {  // uniform branch, almost never taken
        asm volatile("");                     // keeps the exact test out of the common path
        if (near) acos_branch = 4.0 * (double)dot * (double)dot < (double)na * (double)nb;
    }
    float P = cross_norm2<U8>(a, b, na, nb, dot);
    float X = (na * nb) * (1.0f + z);
    float tau = P * rsq_pos<U8>(P * X);
    // the clamp at 0 matters for the ASIN row only (q = 3 dips below 0 next to
    // tau = 0); every ACOS row stays above 1 on [-1, 1/2]
    return acos_branch ? horner4(cf.acos_c, z) : fmaxf(horner4(cf.asin_c, tau), 0.0f);
}

template <bool U8>
__device__ __forceinline__ float angle_minimax(const float4& a, const float4& ra, const float4& b,
                                               const float4& rb, const MinimaxCoef& cf) {
    return angle_minimax_from_dot<U8>(a, ra.w, b, rb.w, dot3(a, b), cf);
}

// Chromaticity numerators a_k sum(b) - b_k sum(a) of float directions, in
// binary64: the channel sums of three binary32 values are exact there (the
// direction is scaled into [1, 2), so a component more than 2^29 below the
// largest is the only case that rounds, at 2^-53), and so are the products
// (24 x at most 27 significant bits); each numerator is then rounded once.
// Rounded binary32 sums and products would leave an absolute error of about
// 2^-24 |a| |b| in a numerator that cancels to |a| |b| B for nearly equal
// chromaticities, i.e. a relative error of 2^-24 / B in B.  The two products
// are rounded separately (no contraction), so swapping a and b negates every
// numerator exactly and the pair term stays bitwise symmetric.
__device__ __forceinline__ float chroma_num2_f64(const float4& a, const float4& b) {
#pragma clang fp contract(off)
    const double a0 = a.x, a1 = a.y, a2 = a.z, b0 = b.x, b1 = b.y, b2 = b.z;
    const double sa = (a0 + a1) + a2, sb = (b0 + b1) + b2;
    const float n0 = (float)(a0 * sb - b0 * sa);
    const float n1 = (float)(a1 * sb - b1 * sa);
    const float n2 = (float)(a2 * sb - b2 * sa);
    return fmaf(n0, n0, fmaf(n1, n1, n2 * n2));
}

// Method 2 (Section 2.2, eq. 7): L2 distance of chromaticities
// |a / sum a - b / sum b| = |a sum b - b sum a| / (sum a sum b).
template <int KIND, bool U8>
__device__ __forceinline__ float chroma_term(const float4& a, float ia, const float4& b, float ib) {
    float Nn;
    if constexpr (U8) {
        // integer numerators, exact in binary32 (cross_diff)
        const float sa = aux_mag<U8>(a.w), sb = aux_mag<U8>(b.w);
        float n0 = cross_diff<U8>(a.x, sb, b.x, sa);
        float n1 = cross_diff<U8>(a.y, sb, b.y, sa);
        float n2 = cross_diff<U8>(a.z, sb, b.z, sa);
        Nn = fmaf(n0, n0, fmaf(n1, n1, n2 * n2));
    } else {
        Nn = chroma_num2_f64(a, b);
    }
    float B = sqrt_raw(Nn) * (ia * ib);
    if (KIND != kBVDF) B = fmaf(kEq10Alpha, B, kEq10Beta);  // eq. (10), Experiment 2
    return B;
}

// The angular term of a pixel with itself, a constant of the variant: the
// cross product and the chromaticity numerators of equal vectors vanish
// exactly (both layouts), so the exact angle is 0, the minimax angle the ASIN
// row at tau = 0 (its constant coefficient, clamped at 0), and the
// chromaticity distance 0 (eq. 10 maps it to its offset).
template <int KIND, int DIST>
__device__ __forceinline__ float self_term(const MinimaxCoef& cf) {
    if (DIST == kExact) return 0.0f;
    if (DIST == kMinimax) return fmaxf(cf.asin_c[0], 0.0f);
    return KIND != kBVDF ? kEq10Beta : 0.0f;
}

// Angular pair term of the chosen variant (float layout, or uint8 with raw.w =
// aux2).
template <int KIND, int DIST, bool U8>
__device__ __forceinline__ float pair_term(const float4& a, const float4& ra, const float4& b,
                                           const float4& rb, const MinimaxCoef& cf,
                                           const AtanCoef& ac) {
    if (DIST == kExact) return angle_exact<U8>(a, b, ac);
    if (DIST == kMinimax) return angle_minimax<U8>(a, ra, b, rb, cf);
    return chroma_term<KIND, U8>(a, ra.w, b, rb.w);
}

// eq. (1) with the L2 norm (Section III), on raw float values.
__device__ __forceinline__ float l2_term(const float4& ra, const float4& rb) {
    float e0 = ra.x - rb.x, e1 = ra.y - rb.y, e2 = ra.z - rb.z;
    return sqrt_raw(fmaf(e0, e0, fmaf(e1, e1, e2 * e2)));
}

// Pair terms of uint8 member a (aux2 ia; a_zero: a is the zero pixel, and
// a_zero_wave the ballot of a_zero over the wave) and neighbour b (aux2 ib): the angular term in th if ANG, the L2 distance of
// eq. (1) in l2 if L2.  EXACT and MINIMAX share the dot product of the
// directions with the L2 term: |x_a - x_b|^2 = |x_a|^2 + |x_b|^2 - 2 x_a.x_b,
// every term an integer exact in binary32.  The zero pixel (direction (1,1,1),
// value 0) breaks the identity (and the raw difference of RGB); lanes with a
// zero pixel take the distance from the other pixel's norm in a branch the
// wave enters only when some lane needs it.
template <int KIND, int DIST, bool ANG, bool L2>
__device__ __forceinline__ void pair_u8(const float4& a, float ia, bool a_zero, uint64_t a_zero_wave,
                                        const float4& b, float ib, const MinimaxCoef& cf,
                                        const AtanCoef& ac, float& th, float& l2) {
    float dot = 0.0f;
    if constexpr (DIST != kRgb) dot = dot3(a, b);
    if constexpr (ANG) {
        if constexpr (DIST == kExact) th = angle_exact_from_dot<true>(a, b, dot, ac);
        else if constexpr (DIST == kMinimax) th = angle_minimax_from_dot<true>(a, ia, b, ib, dot, cf);
        else th = chroma_term<KIND, true>(a, ia, b, ib);
    }
    if constexpr (L2) {
        float l2sq;
        if constexpr (DIST != kRgb) {
            l2sq = fmaf(-2.0f, dot, a.w + b.w);
        } else {
            const float e0 = a.x - b.x, e1 = a.y - b.y, e2 = a.z - b.z;
            l2sq = fmaf(e0, e0, fmaf(e1, e1, e2 * e2));
        }
        const bool b_zero = b.w < 0.0f;
        // a_zero_wave: the lanes whose member a is the zero pixel
        if (__builtin_amdgcn_ballot_w64(b_zero) | a_zero_wave) {
            asm volatile("");  // keeps the fix-up out of the common path
            if (a_zero | b_zero) {
                if constexpr (DIST != kRgb)
                    l2sq = fmaxf(a.w, 0.0f) + fmaxf(b.w, 0.0f);
                else
                    l2sq = (a_zero ? 0.0f : dot3(a, a)) + (b_zero ? 0.0f : dot3(b, b));
            }
        }
        l2 = sqrt_raw(l2sq);
    }
}

// Total order on floats (no NaN) as unsigned keys.
__device__ __forceinline__ uint32_t order_key(float v) {
    uint32_t bits = __float_as_uint(v + 0.0f);  // -0 -> +0
    return (bits & 0x80000000u) ? ~bits : (bits | 0x80000000u);
}

}  // namespace odf
