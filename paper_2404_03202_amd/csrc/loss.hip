// loss.hip -- L1 photometric term of Eq. 17 (lambda = 0) and its gradient,
// plus the small fill kernel used to clear accumulators (a kernel rather
// than hipMemsetAsync, so the sequence stays valid under graph capture).
#include "internal.h"

namespace omnigs {
namespace {

constexpr int kL1Blocks = 1024;
constexpr int kL1Threads = 256;

// Grid-stride pass with a fixed grid: every element lands in the same
// thread's partial on every run, so the reduction order is fixed.
__global__ __launch_bounds__(kL1Threads) void k_l1_partial(const float *image, const float *target, int64_t count,
                                                            float *grad, double *partial) {
    __shared__ double red[kL1Threads];
    const float inv = (float)(1.0 / (double)count);
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kL1Threads + threadIdx.x; i < count;
         i += (int64_t)kL1Blocks * kL1Threads) {
        const float r = image[i] - target[i];
        s += (double)fabsf(r);
        if (grad) grad[i] = r > 0.0f ? inv : (r < 0.0f ? -inv : 0.0f);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kL1Threads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kL1Threads) void k_l1_final(const double *partial, int64_t count, float *loss) {
    __shared__ double red[kL1Threads];
    double s = 0.0;
    for (int k = threadIdx.x; k < kL1Blocks; k += kL1Threads) s += partial[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kL1Threads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(red[0] / (double)count);
}

}  // namespace

size_t l1_scratch_bytes() { return kL1Blocks * sizeof(double); }

hipError_t launch_l1(const float *image, const float *target, int64_t count, float *grad, float *loss, void *scratch,
                     hipStream_t st) {
    double *partial = static_cast<double *>(scratch);
    hipLaunchKernelGGL(k_l1_partial, dim3(kL1Blocks), dim3(kL1Threads), 0, st, image, target, count, grad, partial);
    hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(kL1Threads), 0, st, partial, count, loss);
    return hipGetLastError();
}

}  // namespace omnigs
