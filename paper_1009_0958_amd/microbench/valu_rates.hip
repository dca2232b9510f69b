// valu_rates.hip -- measured issue rates of the instruction classes the
// filter kernels use, and the plain-copy HBM bandwidth, on the current GPU.
// Prints one JSON object.  Used to check the roofline cost model (binary32
// fma/add, transcendentals, binary64 add) and to calibrate byte counters.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>

#define CHECK(x)                                                                   \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                \
            exit(1);                                                               \
        }                                                                          \
    } while (0)

constexpr int kChains = 8;
constexpr int kThreads = 256;

template <int OP>
__global__ void __launch_bounds__(kThreads) rate_kernel(float* out, int iters, float a, float b) {
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = 1.0f + 0.001f * (threadIdx.x + c);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if (OP == 0) x[c] = fmaf(x[c], a, b);                              // fma
            if (OP == 1) x[c] = fmaf(__builtin_amdgcn_rsqf(x[c]), a, b);       // rsq + fma
            if (OP == 2) x[c] = fmaf(__builtin_amdgcn_sqrtf(x[c]), a, b);      // sqrt + fma
            if (OP == 3) x[c] = fmaf(__builtin_amdgcn_logf(x[c]), a, b);       // log + fma
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) rate_f64(double* out, int iters, double a, double b) {
    double x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = 1.0 + 0.001 * (threadIdx.x + c);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = fma(x[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

__global__ void __launch_bounds__(kThreads) copy_kernel(const float4* __restrict__ src,
                                                        float4* __restrict__ dst, size_t n) {
    size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
    size_t stride = (size_t)gridDim.x * kThreads;
    for (; i < n; i += stride) dst[i] = src[i];
}

int main() {
    int dev = 0;
    CHECK(hipSetDevice(dev));
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, dev));
    const int cus = prop.multiProcessorCount;
    const int blocks = cus * 16;
    const int iters = 4096;
    float* out = nullptr;
    double* outd = nullptr;
    CHECK(hipMalloc(&out, sizeof(float) * blocks * kThreads));
    CHECK(hipMalloc(&outd, sizeof(double) * blocks * kThreads));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const double lane_ops = (double)blocks * kThreads * iters * kChains;
    double rates[5];
    for (int op = 0; op < 5; ++op) {
        for (int rep = 0; rep < 2; ++rep) {  // first run warms up
            CHECK(hipEventRecord(e0, 0));
            switch (op) {
            case 0: hipLaunchKernelGGL(rate_kernel<0>, blocks, kThreads, 0, 0, out, iters, 0.999f, 0.001f); break;
            case 1: hipLaunchKernelGGL(rate_kernel<1>, blocks, kThreads, 0, 0, out, iters, 0.999f, 0.5f); break;
            case 2: hipLaunchKernelGGL(rate_kernel<2>, blocks, kThreads, 0, 0, out, iters, 0.999f, 0.5f); break;
            case 3: hipLaunchKernelGGL(rate_kernel<3>, blocks, kThreads, 0, 0, out, iters, 0.5f, 2.0f); break;
            default: hipLaunchKernelGGL(rate_f64, blocks, kThreads, 0, 0, outd, iters, 0.999, 0.001); break;
            }
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(e1, 0));
            CHECK(hipEventSynchronize(e1));
        }
        float ms = 0.0f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        rates[op] = lane_ops / (ms * 1e-3);  // loop bodies per second (lane level)
    }
    // plain copy of 1 GiB: bytes read + written per second
    const size_t n = (size_t)1 << 26;  // float4 elements = 1 GiB
    float4 *src = nullptr, *dst = nullptr;
    CHECK(hipMalloc(&src, n * sizeof(float4)));
    CHECK(hipMalloc(&dst, n * sizeof(float4)));
    CHECK(hipMemset(src, 0, n * sizeof(float4)));
    float cms = 0.0f;
    for (int rep = 0; rep < 3; ++rep) {
        CHECK(hipEventRecord(e0, 0));
        hipLaunchKernelGGL(copy_kernel, cus * 32, kThreads, 0, 0, src, dst, n);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1, 0));
        CHECK(hipEventSynchronize(e1));
        CHECK(hipEventElapsedTime(&cms, e0, e1));
    }
    const double fma = rates[0];
    printf("{\"device\": \"%s\", \"cus\": %d, \"clock_mhz\": %d, "
           "\"fma_f32_lane_per_s\": %.4e, \"rsq_plus_fma_lane_per_s\": %.4e, "
           "\"sqrt_plus_fma_lane_per_s\": %.4e, \"log_plus_fma_lane_per_s\": %.4e, "
           "\"fma_f64_lane_per_s\": %.4e, \"rsq_cost_in_fma\": %.3f, \"sqrt_cost_in_fma\": %.3f, "
           "\"log_cost_in_fma\": %.3f, \"copy_bytes\": %zu, \"copy_ms\": %.4f, "
           "\"copy_GBps\": %.1f}\n",
           prop.name, cus, prop.clockRate / 1000, rates[0], rates[1], rates[2], rates[3], rates[4],
           fma / rates[1] - 1.0, fma / rates[2] - 1.0, fma / rates[3] - 1.0,
           2 * n * sizeof(float4), cms, 2.0 * n * sizeof(float4) / (cms * 1e-3) / 1e9);
    CHECK(hipFree(src));
    CHECK(hipFree(dst));
    CHECK(hipFree(out));
    CHECK(hipFree(outd));
    return 0;
}
