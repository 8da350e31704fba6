// loss.hip -- the photometric loss of Eq. 17 and its gradient: the L1 term,
// and L = (1 - lambda) L1 + lambda (1 - SSIM) with SSIM on 11x11 Gaussian
// windows (sigma 1.5) over zero-padded images.
#include "internal.h"

#include <cmath>

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

// ------------------------------------------------------------------ SSIM
// One workgroup per 16x16 tile and channel, fused forward and backward.  The
// gradient at pixel p gathers the windows centred at q with |q - p| <= 5
// (the window is symmetric), so the workgroup needs the SSIM partials on the
// 26x26 centres around its tile, hence the window statistics there, hence x
// and y on a 36x36 halo: every step is a separable 11-tap pass in LDS.  Only
// x, y are read and dL/dx written; per-tile partial sums of S and |x - y|
// go to a partials array reduced in a fixed order.
constexpr int kSsimT = 16;              // output tile edge
constexpr int kSsimR = 5;               // window radius (11 taps)
constexpr int kSsimC = kSsimT + 2 * kSsimR;  // 26: centres whose window reaches the tile
constexpr int kSsimH = kSsimC + 2 * kSsimR;  // 36: pixels those windows read
constexpr int kSsimThreads = 256;
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct SsimArgs {
    const float *x, *y;
    float *grad;      // may be null
    double *partial;  // [tiles * channels][2]: sum S, sum |x - y| over the tile
    int width, height, tiles_x;
    float w1[2 * kSsimR + 1];  // normalised 1D Gaussian, sigma 1.5
    float lambda, inv_n;
};

__global__ __launch_bounds__(kSsimThreads) void k_ssim(SsimArgs a) {
    __shared__ float X[kSsimH][kSsimH], Y[kSsimH][kSsimH];
    __shared__ float Hs[5][kSsimH][kSsimC];    // horizontal sums: x, y, xx, yy, xy
    __shared__ float Mp[5][kSsimC][kSsimC];    // partials at the centres: A, B, B mu_x, C, C mu_y
    __shared__ float H2[5][kSsimC][kSsimT];    // their horizontal sums
    __shared__ double red[2][kSsimThreads];
    const int c = blockIdx.z;
    const int tx0 = blockIdx.x * kSsimT, ty0 = blockIdx.y * kSsimT;
    const int64_t plane = (int64_t)a.width * a.height;
    const float *xs = a.x + c * plane, *ys = a.y + c * plane;
    const int tid = threadIdx.x;
    // 1. halo, zero outside the image
    for (int k = tid; k < kSsimH * kSsimH; k += kSsimThreads) {
        const int r = k / kSsimH, q = k % kSsimH;
        const int gy = ty0 - 2 * kSsimR + r, gx = tx0 - 2 * kSsimR + q;
        const bool in = gy >= 0 && gy < a.height && gx >= 0 && gx < a.width;
        X[r][q] = in ? xs[(int64_t)gy * a.width + gx] : 0.0f;
        Y[r][q] = in ? ys[(int64_t)gy * a.width + gx] : 0.0f;
    }
    __syncthreads();
    // 2. horizontal window sums for every halo row at the 26 centre columns
    for (int k = tid; k < kSsimH * kSsimC; k += kSsimThreads) {
        const int r = k / kSsimC, q = k % kSsimC;
        float sx = 0.0f, sy = 0.0f, sxx = 0.0f, syy = 0.0f, sxy = 0.0f;
#pragma unroll
        for (int t = 0; t <= 2 * kSsimR; ++t) {
            const float w = a.w1[t], xv = X[r][q + t], yv = Y[r][q + t];
            sx = __builtin_fmaf(w, xv, sx);
            sy = __builtin_fmaf(w, yv, sy);
            sxx = __builtin_fmaf(w, xv * xv, sxx);
            syy = __builtin_fmaf(w, yv * yv, syy);
            sxy = __builtin_fmaf(w, xv * yv, sxy);
        }
        Hs[0][r][q] = sx;
        Hs[1][r][q] = sy;
        Hs[2][r][q] = sxx;
        Hs[3][r][q] = syy;
        Hs[4][r][q] = sxy;
    }
    __syncthreads();
    // 3. vertical sums: statistics, S and its partials at the 26x26 centres
    double s_sum = 0.0, l1_sum = 0.0;
    for (int k = tid; k < kSsimC * kSsimC; k += kSsimThreads) {
        const int r = k / kSsimC, q = k % kSsimC;
        const int gy = ty0 - kSsimR + r, gx = tx0 - kSsimR + q;
        float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t <= 2 * kSsimR; ++t) {
            const float w = a.w1[t];
#pragma unroll
            for (int f = 0; f < 5; ++f) m[f] = __builtin_fmaf(w, Hs[f][r + t][q], m[f]);
        }
        float A = 0.0f, Bv = 0.0f, Cv = 0.0f, mx = 0.0f, my = 0.0f;
        if (gy >= 0 && gy < a.height && gx >= 0 && gx < a.width) {
            mx = m[0];
            my = m[1];
            const float vxx = m[2] - mx * mx, vyy = m[3] - my * my, vxy = m[4] - mx * my;
            const float n1 = 2.0f * mx * my + kC1, n2 = 2.0f * vxy + kC2;
            const float d1 = mx * mx + my * my + kC1, d2 = vxx + vyy + kC2;
            const float inv = 1.0f / (d1 * d2);
            const float S = n1 * n2 * inv;
            A = 2.0f * my * n2 * inv - S * 2.0f * mx / d1;  // dS/dmu_x
            Bv = -S / d2;                                     // dS/ds_xx
            Cv = 2.0f * n1 * inv;                             // dS/ds_xy
            // the tile's own centres carry the loss
            if (r >= kSsimR && r < kSsimR + kSsimT && q >= kSsimR && q < kSsimR + kSsimT) {
                s_sum += (double)S;
                l1_sum += (double)fabsf(X[r + kSsimR][q + kSsimR] - Y[r + kSsimR][q + kSsimR]);
            }
        }
        Mp[0][r][q] = A;
        Mp[1][r][q] = Bv;
        Mp[2][r][q] = Bv * mx;
        Mp[3][r][q] = Cv;
        Mp[4][r][q] = Cv * my;
    }
    red[0][tid] = s_sum;
    red[1][tid] = l1_sum;
    __syncthreads();
    // 4. horizontal sums of the partials at the 16 output columns
    for (int k = tid; k < kSsimC * kSsimT; k += kSsimThreads) {
        const int r = k / kSsimT, q = k % kSsimT;
        float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t <= 2 * kSsimR; ++t) {
            const float w = a.w1[t];
#pragma unroll
            for (int f = 0; f < 5; ++f) m[f] = __builtin_fmaf(w, Mp[f][r][q + t], m[f]);
        }
#pragma unroll
        for (int f = 0; f < 5; ++f) H2[f][r][q] = m[f];
    }
    for (int off = kSsimThreads / 2; off > 0; off >>= 1) {
        __syncthreads();
        if (tid < off) {
            red[0][tid] += red[0][tid + off];
            red[1][tid] += red[1][tid + off];
        }
    }
    __syncthreads();
    const int64_t blk = ((int64_t)c * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    if (tid == 0) {
        a.partial[2 * blk] = red[0][0];
        a.partial[2 * blk + 1] = red[1][0];
    }
    if (!a.grad) return;
    // 5. vertical sums and the gradient at the tile's pixels
    {
        const int r = tid / kSsimT, q = tid % kSsimT;
        const int gy = ty0 + r, gx = tx0 + q;
        if (gy >= a.height || gx >= a.width) return;
        float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t <= 2 * kSsimR; ++t) {
            const float w = a.w1[t];
#pragma unroll
            for (int f = 0; f < 5; ++f) m[f] = __builtin_fmaf(w, H2[f][r + t][q], m[f]);
        }
        const float xv = X[r + 2 * kSsimR][q + 2 * kSsimR], yv = Y[r + 2 * kSsimR][q + 2 * kSsimR];
        // d S_sum / d x_p = G*A + 2 x_p G*B - 2 G*(B mu_x) + y_p G*C - G*(C mu_y)
        const float dS = m[0] + 2.0f * xv * m[1] - 2.0f * m[2] + yv * m[3] - m[4];
        const float d = xv - yv;
        const float sgn = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
        a.grad[c * plane + (int64_t)gy * a.width + gx] = a.inv_n * ((1.0f - a.lambda) * sgn - a.lambda * dS);
    }
}

// loss = (1 - lambda) sum|x - y| / N + lambda (1 - sum S / N), in a fixed order
__global__ __launch_bounds__(256) void k_ssim_final(const double *partial, int64_t blocks, double n, double lambda,
                                                    float *loss) {
    __shared__ double red[2][256];
    double s = 0.0, l = 0.0;
    for (int64_t k = threadIdx.x; k < blocks; k += 256) {
        s += partial[2 * k];
        l += partial[2 * k + 1];
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = l;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)((1.0 - lambda) * red[1][0] / n + lambda * (1.0 - red[0][0] / n));
}

}  // namespace

size_t ssim_scratch_bytes(int channels, int height, int width) {
    const int64_t tiles = (int64_t)((width + kSsimT - 1) / kSsimT) * ((height + kSsimT - 1) / kSsimT) * channels;
    return (size_t)tiles * 2 * sizeof(double);
}

hipError_t launch_photometric(const float *image, const float *target, int channels, int height, int width,
                              float lambda, float *grad, float *loss, void *scratch, hipStream_t st) {
    SsimArgs a{};
    a.x = image;
    a.y = target;
    a.grad = grad;
    a.partial = static_cast<double *>(scratch);
    a.width = width;
    a.height = height;
    a.tiles_x = (width + kSsimT - 1) / kSsimT;
    double g[2 * kSsimR + 1], sum = 0.0;
    for (int t = 0; t <= 2 * kSsimR; ++t) {
        const double d = t - kSsimR;
        g[t] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        sum += g[t];
    }
    for (int t = 0; t <= 2 * kSsimR; ++t) a.w1[t] = (float)(g[t] / sum);
    const double n = (double)channels * height * width;
    a.lambda = lambda;
    a.inv_n = (float)(1.0 / n);
    const dim3 grid((unsigned)a.tiles_x, (unsigned)((height + kSsimT - 1) / kSsimT), (unsigned)channels);
    hipLaunchKernelGGL(k_ssim, grid, dim3(kSsimThreads), 0, st, a);
    const int64_t blocks = (int64_t)grid.x * grid.y * grid.z;
    hipLaunchKernelGGL(k_ssim_final, dim3(1), dim3(256), 0, st, a.partial, blocks, n, (double)lambda, loss);
    return hipGetLastError();
}

size_t l1_scratch_bytes() { return kL1Blocks * sizeof(double); }

hipError_t launch_l1(const float *image, const float *target, int64_t count, float *grad, float *loss, void *scratch,
                     hipStream_t st) {
    double *partial = static_cast<double *>(scratch);
    hipLaunchKernelGGL(k_l1_partial, dim3(kL1Blocks), dim3(kL1Threads), 0, st, image, target, count, grad, partial);
    hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(kL1Threads), 0, st, partial, count, loss);
    return hipGetLastError();
}

}  // namespace omnigs
