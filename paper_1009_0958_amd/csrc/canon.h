// canon.h -- canonical direction of a uint8 pixel: the colour divided by the
// greatest common divisor of its three channels.
//
// The angle of eq. (2) and the chromaticity of eq. (7) depend on a pixel only
// through its direction, so x and k x (k > 0) give every pair term the same
// value.  Evaluated on the raw integer vectors, rounding tells such collinear
// colours apart by an ulp, and a window whose smallest aggregates belong to
// collinear colours of different brightness picks whichever rounded lowest.
// Taking every pixel's direction as x / gcd(x) makes collinear colours one
// integer vector: their pair terms, aggregates and objectives are then equal
// bit for bit, the tie goes to the lowest member index, and the exact integer
// arithmetic of the uint8 pair terms is kept (the canonical components are
// integers no larger than the raw ones).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace odf {

// gcd(a, b) for a, b in [0, 255], built at compile time: the lower triangle row
// by row from gcd(a, b) = gcd(b, a mod b) (an entry of an earlier row's lower
// triangle), then the upper triangle by symmetry; gcd(a, 0) = a.
struct GcdTable {
    uint8_t g[256 * 256];
    constexpr GcdTable() : g() {
        for (int a = 0; a < 256; ++a) {
            g[a * 256] = (uint8_t)a;
            for (int b = 1; b <= a; ++b) g[a * 256 + b] = g[b * 256 + a % b];
        }
        for (int a = 0; a < 256; ++a)
            for (int b = a + 1; b < 256; ++b) g[a * 256 + b] = g[b * 256 + a];
    }
};
static_assert(GcdTable().g[12 * 256 + 18] == 6 && GcdTable().g[255 * 256 + 0] == 255 &&
                  GcdTable().g[97 * 256 + 89] == 1,
              "gcd table");

// 64 KiB in device global memory (read through the caches), one copy per
// translation unit that uses it.
__device__ const GcdTable kGcdTable;

// The canonical direction of the uint8 pixel (c0, c1, c2) as exact integers in
// binary32; the zero pixel gives gcd 0 and NaN components, which the caller
// replaces by its own convention.  x / g is an integer at most 255, and
// x * rcp(g) lies within 255 * 2^-22 of it, so rounding to the nearest integer
// gives it exactly.
__device__ __forceinline__ void canonical_direction(uint32_t c0, uint32_t c1, uint32_t c2,
                                                    float& d0, float& d1, float& d2) {
    const uint32_t g01 = kGcdTable.g[c0 * 256 + c1];
    const uint32_t g = kGcdTable.g[g01 * 256 + c2];
    const float r = __builtin_amdgcn_rcpf((float)g);
    d0 = rintf((float)c0 * r);
    d1 = rintf((float)c1 * r);
    d2 = rintf((float)c2 * r);
}

}  // namespace odf
