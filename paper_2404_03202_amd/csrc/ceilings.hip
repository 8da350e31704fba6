// ceilings.hip -- measured ceilings of the chip for the rasterizer's bounds:
// the FP32 FMA issue rate without packed math (the blends' arithmetic), the
// exp2 rate (one per evaluated pixel-instance pair), the rate of scattered
// float atomics into a buffer the size of the backward's accumulators, and
// plain copy bandwidth (the HBM-bound stages).  Each is one kernel timed
// with HIP events on the caller's stream; the kernels store nothing except
// behind a runtime flag the host never sets (the FMA and exp chains), their
// atomics, or the copy itself.
#include "internal.h"

namespace omnigs {
namespace {

constexpr int kCeilThreads = 256;
constexpr int kChains = 16;   // independent chains per lane: hides the ALU latency
constexpr int kCeilIters = 1024;

__global__ __launch_bounds__(kCeilThreads) void k_ceiling_fma(float x, float y, int never, float *sink) {
    float a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = (float)(threadIdx.x + c);
    for (int it = 0; it < kCeilIters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = __builtin_fmaf(a[c], x, y);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += a[c];
    if (never) sink[blockIdx.x * kCeilThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kCeilThreads) void k_ceiling_exp(float scale, int never, float *sink) {
    float a[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = scale * (float)(threadIdx.x + c);
    for (int it = 0; it < kCeilIters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = __builtin_amdgcn_exp2f(-a[c]);  // stays in [0.5, 1]
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += a[c];
    if (never) sink[blockIdx.x * kCeilThreads + threadIdx.x] = s;
}

// kAtomicsPerLane float atomics per lane at hashed word addresses in
// [0, words): the scatter of the backward's per-Gaussian accumulators.
constexpr int kAtomicsPerLane = 16;
__global__ __launch_bounds__(kCeilThreads) void k_ceiling_atomic(float *buf, uint32_t words) {
    const uint32_t i = blockIdx.x * kCeilThreads + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kAtomicsPerLane; ++k) {
        uint32_t h = (i * kAtomicsPerLane + k) * 2654435761u;
        h ^= h >> 15;
        atomicAdd(buf + (uint32_t)(((uint64_t)h * words) >> 32), 1.0f);
    }
}

__global__ __launch_bounds__(kCeilThreads) void k_ceiling_copy(const float4 *src, float4 *dst, int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * kCeilThreads;
    for (int64_t i = (int64_t)blockIdx.x * kCeilThreads + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

}  // namespace

hipError_t measure_ceilings(float *atomic_buf, uint32_t atomic_words, const float *copy_src, float *copy_dst,
                            int64_t copy_bytes, int repeats, double ms[4], double work[4], hipStream_t st) {
    hipEvent_t e0, e1;
    hipError_t err;
    if ((err = hipEventCreate(&e0)) != hipSuccess) return err;
    if ((err = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return err;
    }
    // 8192 blocks of 4 waves: 128 waves per CU over the 256 CUs
    const unsigned blocks = 8192;
    const int64_t lanes = (int64_t)blocks * kCeilThreads;
    const int64_t n4 = copy_bytes / 16;
    auto launch = [&](int k) {
        switch (k) {
        case 0: hipLaunchKernelGGL(k_ceiling_fma, dim3(blocks), dim3(kCeilThreads), 0, st, 0.999f, 1e-3f, 0, nullptr); break;
        case 1: hipLaunchKernelGGL(k_ceiling_exp, dim3(blocks), dim3(kCeilThreads), 0, st, 1e-3f, 0, nullptr); break;
        case 2: hipLaunchKernelGGL(k_ceiling_atomic, dim3(blocks), dim3(kCeilThreads), 0, st, atomic_buf, atomic_words); break;
        default:
            hipLaunchKernelGGL(k_ceiling_copy, dim3(4096), dim3(kCeilThreads), 0, st,
                               reinterpret_cast<const float4 *>(copy_src), reinterpret_cast<float4 *>(copy_dst), n4);
        }
    };
    const double per_launch[4] = {(double)lanes * kChains * kCeilIters * 2.0,  // FLOP (FMA = 2)
                                  (double)lanes * kChains * kCeilIters,        // exp2 results
                                  (double)lanes * kAtomicsPerLane,             // atomics
                                  (double)n4 * 32.0};                          // bytes read + written
    for (int k = 0; k < 4 && err == hipSuccess; ++k) {
        ms[k] = 0.0;
        work[k] = 0.0;
        if ((k == 2 && (!atomic_buf || atomic_words == 0)) || (k == 3 && (!copy_src || !copy_dst || n4 == 0))) continue;
        launch(k);  // warm-up
        if ((err = hipGetLastError()) != hipSuccess) break;
        if ((err = hipEventRecord(e0, st)) != hipSuccess) break;
        for (int r = 0; r < repeats; ++r) launch(k);
        if ((err = hipGetLastError()) != hipSuccess) break;
        if ((err = hipEventRecord(e1, st)) != hipSuccess) break;
        if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
        float t = 0.0f;
        if ((err = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) break;
        ms[k] = (double)t / repeats;
        work[k] = per_launch[k];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return err;
}

}  // namespace omnigs
