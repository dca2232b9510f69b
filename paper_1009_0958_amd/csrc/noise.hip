// noise.hip -- the correlated impulsive noise model of eq. (8) (Section III)
// and the MAE / PSNR effectiveness measures, on the GPU.
//
// Noise: every pixel draws one Philox4x32-10 block (Salmon, Moraes, Dror and
// Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011) with the flat
// pixel index as counter (low word, high word, 0, 0) and the 64-bit seed as
// key.  Word 0 decides corruption (u0 < floor(phi 2^32)), word 1 the channel
// pattern against the cumulative thresholds of phi_1, phi_2, phi_3 (red only,
// green only, blue only, else all three), and the bytes of word 2 are the
// random vector r (uniform in {0..255}^3).  Memory-bound: 3 bytes in and out
// per pixel.
//
// Quality: per image, exact 64-bit integer sums of |y - o| and (y - o)^2 over
// the 3MN channel values (order-independent, so atomics keep them exact), then
// MAE = S1 / 3MN and PSNR = 10 log10(255^2 3MN / S2) in binary64.
#include <algorithm>

#include "odf.h"
#include "odf_internal.h"

namespace odf {

namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint32_t hi0 = __umulhi(kPhiloxM0, c[0]), lo0 = kPhiloxM0 * c[0];
        const uint32_t hi1 = __umulhi(kPhiloxM1, c[2]), lo1 = kPhiloxM1 * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

struct NoiseParams {
    const uint8_t* clean;
    uint8_t* noisy;
    long long npix;
    uint64_t t_hit;          // corrupt iff u0 < t_hit (0 .. 2^32)
    uint64_t t_pat[3];       // cumulative pattern thresholds
    uint32_t key0, key1;
};

// Noise of one pixel (eq. 8): the Philox4x32-10 block of counter i decides
// whether the pixel is hit, which channels change, and their random bytes.
__device__ __forceinline__ void noise_pixel(const NoiseParams& prm, long long i, uint8_t& o0,
                                            uint8_t& o1, uint8_t& o2) {
    uint32_t c[4] = {(uint32_t)i, (uint32_t)((unsigned long long)i >> 32), 0u, 0u};
    philox4x32_10(c, prm.key0, prm.key1);
    if ((uint64_t)c[0] < prm.t_hit) {
        const uint64_t u1 = c[1];
        const int pat = u1 < prm.t_pat[0] ? 0 : u1 < prm.t_pat[1] ? 1 : u1 < prm.t_pat[2] ? 2 : 3;
        if (pat == 0 || pat == 3) o0 = (uint8_t)(c[2] & 0xffu);
        if (pat == 1 || pat == 3) o1 = (uint8_t)((c[2] >> 8) & 0xffu);
        if (pat == 2 || pat == 3) o2 = (uint8_t)((c[2] >> 16) & 0xffu);
    }
}

// VEC: both buffers 4-byte aligned; a thread takes four pixels (twelve bytes,
// three words) per step and the last npix % 4 pixels one by one.  Each pixel
// keeps its own counter, so the output does not depend on the form.
template <bool VEC>
__global__ void __launch_bounds__(256) noise_kernel(NoiseParams prm) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long first = 0;  // first pixel of the one-by-one loop
    if (VEC) {
        const long long nq = prm.npix / 4;
        const uint32_t* s = reinterpret_cast<const uint32_t*>(prm.clean);
        uint32_t* d = reinterpret_cast<uint32_t*>(prm.noisy);
        for (long long q = t0; q < nq; q += stride) {
            uint32_t w[3] = {s[3 * q], s[3 * q + 1], s[3 * q + 2]};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                // pixel k holds bytes 3k .. 3k + 2 of the twelve (little-endian words)
                uint8_t o[3];
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    o[j] = (uint8_t)(w[(3 * k + j) / 4] >> (8 * ((3 * k + j) % 4)));
                noise_pixel(prm, 4 * q + k, o[0], o[1], o[2]);
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int sh = 8 * ((3 * k + j) % 4);
                    uint32_t& v = w[(3 * k + j) / 4];
                    v = (v & ~(0xffu << sh)) | ((uint32_t)o[j] << sh);
                }
            }
            d[3 * q] = w[0];
            d[3 * q + 1] = w[1];
            d[3 * q + 2] = w[2];
        }
        first = nq * 4;
    }
    for (long long i = first + t0; i < prm.npix; i += stride) {
        const uint8_t* s = prm.clean + 3 * i;
        uint8_t o0 = s[0], o1 = s[1], o2 = s[2];
        noise_pixel(prm, i, o0, o1, o2);
        uint8_t* d = prm.noisy + 3 * i;
        d[0] = o0;
        d[1] = o1;
        d[2] = o2;
    }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void add_diffs(uint32_t a, uint32_t b, unsigned long long& s1,
                                          unsigned long long& s2) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int d = (int)((a >> (8 * k)) & 0xffu) - (int)((b >> (8 * k)) & 0xffu);
        s1 += (unsigned)(d < 0 ? -d : d);
        s2 += (unsigned)(d * d);
    }
}

struct QualityParams {
    const uint8_t* y;
    const uint8_t* ref;
    long long nbytes;             // 3MN per image
    unsigned long long* sums;     // 2 per image: S1, S2
    double* mae;
    double* psnr;
    int B;
};

// One image per blockIdx.y.  VEC: every image starts 16-byte aligned in both
// arrays and 3MN is a multiple of 16, so the image is read as uint4 chunks.
template <bool VEC>
__global__ void __launch_bounds__(256) quality_kernel(QualityParams prm) {
    const int b = blockIdx.y;
    const uint8_t* y = prm.y + (size_t)b * prm.nbytes;
    const uint8_t* r = prm.ref + (size_t)b * prm.nbytes;
    unsigned long long s1 = 0, s2 = 0;
    const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    if (VEC) {
        const uint4* yv = reinterpret_cast<const uint4*>(y);
        const uint4* rv = reinterpret_cast<const uint4*>(r);
        for (long long i = t0; i < prm.nbytes / 16; i += stride) {
            const uint4 a = yv[i], c = rv[i];
            add_diffs(a.x, c.x, s1, s2);
            add_diffs(a.y, c.y, s1, s2);
            add_diffs(a.z, c.z, s1, s2);
            add_diffs(a.w, c.w, s1, s2);
        }
    } else {
        for (long long i = t0; i < prm.nbytes; i += stride) {
            const int d = (int)y[i] - (int)r[i];
            s1 += (unsigned)(d < 0 ? -d : d);
            s2 += (unsigned)(d * d);
        }
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    __shared__ unsigned long long part[2][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        part[0][wave] = s1;
        part[1][wave] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long a = part[0][0] + part[0][1] + part[0][2] + part[0][3];
        const unsigned long long c = part[1][0] + part[1][1] + part[1][2] + part[1][3];
        atomicAdd(&prm.sums[2 * b], a);
        atomicAdd(&prm.sums[2 * b + 1], c);
    }
}

__global__ void quality_clear(unsigned long long* sums, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) sums[i] = 0ull;
}

__global__ void quality_finish(QualityParams prm) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= prm.B) return;
    const double n = (double)prm.nbytes;
    const unsigned long long s1 = prm.sums[2 * b], s2 = prm.sums[2 * b + 1];
    prm.mae[b] = (double)s1 / n;
    prm.psnr[b] = s2 == 0 ? __builtin_huge_val() : 10.0 * log10(255.0 * 255.0 * n / (double)s2);
}

uint64_t threshold32(double p) {  // floor(p 2^32), p in [0, 1]
    const double t = p * 4294967296.0;
    return t >= 4294967296.0 ? 4294967296ull : (uint64_t)t;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

}  // namespace

}  // namespace odf

extern "C" {

int odf_noise_eq8_u8(const uint8_t* clean, uint8_t* noisy, int B, int M, int N, double phi,
                     double phi_r, double phi_g, double phi_b, uint64_t seed, void* stream) {
    using odf::set_error;
    if (!clean || !noisy) return set_error(ODF_EINVAL, "noise: clean/noisy is NULL");
    if (B < 1 || M < 1 || N < 1 || (long long)B * M * N >= (1ll << 40))
        return set_error(ODF_EINVAL, "noise: sizes out of range");
    if (!(phi >= 0.0 && phi <= 1.0) || !(phi_r >= 0.0) || !(phi_g >= 0.0) || !(phi_b >= 0.0) ||
        !(phi_r + phi_g + phi_b <= 1.0))
        return set_error(ODF_EINVAL,
                         "noise: phi must lie in [0, 1] and phi_r, phi_g, phi_b >= 0 with sum <= 1");
    const long long npix = (long long)B * M * N;
    if (clean != noisy && odf::overlap(clean, 3 * npix, noisy, 3 * npix))
        return set_error(ODF_EINVAL, "noise: noisy partially overlaps clean");
    odf::NoiseParams prm{};
    prm.clean = clean;
    prm.noisy = noisy;
    prm.npix = npix;
    prm.t_hit = odf::threshold32(phi);
    prm.t_pat[0] = odf::threshold32(phi_r);
    prm.t_pat[1] = odf::threshold32(phi_r + phi_g);
    prm.t_pat[2] = odf::threshold32(phi_r + phi_g + phi_b);
    prm.key0 = (uint32_t)seed;
    prm.key1 = (uint32_t)(seed >> 32);
    // four pixels per thread when both buffers are 4-byte aligned
    const bool vec =
        ((reinterpret_cast<uintptr_t>(clean) | reinterpret_cast<uintptr_t>(noisy)) & 3) == 0;
    const long long work = vec ? (npix + 3) / 4 : npix;
    const long long blocks = std::min<long long>((work + 255) / 256, 1 << 16);
    if (vec)
        hipLaunchKernelGGL(odf::noise_kernel<true>, dim3((unsigned)blocks), dim3(256), 0,
                           static_cast<hipStream_t>(stream), prm);
    else
        hipLaunchKernelGGL(odf::noise_kernel<false>, dim3((unsigned)blocks), dim3(256), 0,
                           static_cast<hipStream_t>(stream), prm);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ODF_EHIP, "noise launch: %s", hipGetErrorString(e));
    return ODF_OK;
}

size_t odf_quality_workspace(int B) { return B < 1 ? 0 : (size_t)B * 2 * sizeof(uint64_t); }

int odf_quality_u8(const uint8_t* y, const uint8_t* ref, int B, int M, int N, double* mae,
                   double* psnr, void* workspace, size_t workspace_bytes, void* stream) {
    using odf::set_error;
    if (!y || !ref || !mae || !psnr || !workspace)
        return set_error(ODF_EINVAL, "quality: a pointer is NULL");
    if (B < 1 || B > 65535 || M < 1 || N < 1 || (long long)B * M * N >= (1ll << 40))
        return set_error(ODF_EINVAL, "quality: sizes out of range");
    if (workspace_bytes < odf_quality_workspace(B))
        return set_error(ODF_EINVAL, "quality: workspace smaller than odf_quality_workspace(B)");
    if ((reinterpret_cast<uintptr_t>(workspace) & 7) != 0)
        return set_error(ODF_EINVAL, "quality: workspace must be 8-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    odf::QualityParams prm{};
    prm.y = y;
    prm.ref = ref;
    prm.nbytes = 3ll * M * N;
    prm.sums = static_cast<unsigned long long*>(workspace);
    prm.mae = mae;
    prm.psnr = psnr;
    prm.B = B;
    const bool vec = ((reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(ref)) & 15) == 0 &&
                     prm.nbytes % 16 == 0;
    const long long units = vec ? prm.nbytes / 16 : prm.nbytes;
    const unsigned bx = (unsigned)std::max<long long>(1, std::min<long long>((units + 1023) / 1024, 512));
    hipLaunchKernelGGL(odf::quality_clear, dim3(1), dim3(256), 0, s, prm.sums, 2 * B);
    if (vec)
        hipLaunchKernelGGL(odf::quality_kernel<true>, dim3(bx, B), dim3(256), 0, s, prm);
    else
        hipLaunchKernelGGL(odf::quality_kernel<false>, dim3(bx, B), dim3(256), 0, s, prm);
    hipLaunchKernelGGL(odf::quality_finish, dim3((B + 255) / 256), dim3(256), 0, s, prm);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(ODF_EHIP, "quality launch: %s", hipGetErrorString(e));
    return ODF_OK;
}

}  // extern "C"
