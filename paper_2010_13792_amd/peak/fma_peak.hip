// fma_peak.hip -- issue-rate microbenchmark for the VALU rooflines.
//
// Every thread runs independent chains of fused multiply-adds (FP32 with
// packed FP32 instructions disabled, as in the library, and FP64) over a
// grid of 8 workgroups of 256 threads per compute unit, and writes one
// value, so the loop cannot be removed.  Prints one JSON line with the best
// of three timed launches per variant (flops = 2 per FMA).
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kUnroll = 16;

template <class R, int C>
__global__ void __launch_bounds__(256) k_fma(R* __restrict__ out, R a, R b, int iters) {
    R x[C];
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = (R)(threadIdx.x + c) * (R)1e-3;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int c = 0; c < C; ++c) x[c] = __builtin_fma(x[c], a, b);
    }
    R s = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) s += x[c];
    out[blockIdx.x * (size_t)blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_fma32(float* __restrict__ out, float a, float b, int iters) {
    float x[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) x[c] = (float)(threadIdx.x + c) * 1e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int c = 0; c < 16; ++c) x[c] = __builtin_fmaf(x[c], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 16; ++c) s += x[c];
    out[blockIdx.x * (size_t)blockDim.x + threadIdx.x] = s;
}

#define CK(x)                                                                  \
    do {                                                                       \
        hipError_t e_ = (x);                                                   \
        if (e_ != hipSuccess) {                                                \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));       \
            return 1;                                                          \
        }                                                                      \
    } while (0)

}  // namespace

int main() {
    int dev = 0, cus = 0;
    CK(hipGetDevice(&dev));
    CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = cus * 8, threads = 256, iters = 400;
    const size_t nthr = (size_t)blocks * threads;
    float* o32 = nullptr;
    double* o64 = nullptr;
    CK(hipMalloc(&o32, nthr * sizeof(float)));
    CK(hipMalloc(&o64, nthr * sizeof(double)));
    hipEvent_t e0, e1;
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    double best32 = 0.0, best64 = 0.0;
    for (int rep = 0; rep < 4; ++rep) {   // the first round only warms up
        float ms = 0.f;
        CK(hipEventRecord(e0));
        hipLaunchKernelGGL(k_fma32, dim3(blocks), dim3(threads), 0, 0, o32, 0.9999999f, 1e-7f, iters);
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        CK(hipGetLastError());
        CK(hipEventElapsedTime(&ms, e0, e1));
        const double f32 = (double)nthr * iters * kUnroll * 16 * 2 / (ms * 1e-3) / 1e12;
        CK(hipEventRecord(e0));
        hipLaunchKernelGGL((k_fma<double, 8>), dim3(blocks), dim3(threads), 0, 0, o64, 0.9999999, 1e-7, iters);
        CK(hipEventRecord(e1));
        CK(hipEventSynchronize(e1));
        CK(hipGetLastError());
        CK(hipEventElapsedTime(&ms, e0, e1));
        const double f64 = (double)nthr * iters * kUnroll * 8 * 2 / (ms * 1e-3) / 1e12;
        if (rep > 0) {
            best32 = f32 > best32 ? f32 : best32;
            best64 = f64 > best64 ? f64 : best64;
        }
    }
    float h = 0.f;
    CK(hipMemcpy(&h, o32, sizeof(h), hipMemcpyDeviceToHost));
    std::printf("{\"fp32_fma_tflops\": %.2f, \"fp64_fma_tflops\": %.2f, \"compute_units\": %d, \"check\": %g}\n",
                best32, best64, cus, (double)h);
    CK(hipFree(o32));
    CK(hipFree(o64));
    return 0;
}
