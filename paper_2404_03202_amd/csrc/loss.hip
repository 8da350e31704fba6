// loss.hip -- the photometric loss of Eq. 17 and its gradient: the L1 term,
// and L = (1 - lambda) L1 + lambda (1 - SSIM) with SSIM on 11x11 Gaussian
// windows (sigma 1.5) over zero-padded images.
#include "internal.h"

#include <cmath>

namespace omnigs {
namespace {

constexpr int kL1Blocks = 1024;
constexpr int kL1Threads = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Grid-stride pass with a fixed grid: every element lands in the same
// thread's partial on every run, so the reduction order is fixed.
// kVec: image, target and grad are 16-byte aligned and the grid strides over
// float4 groups (the last count % 4 elements by the first threads); each
// thread issues the loads of kL1Unroll strided groups before it uses them
// (and adds them in the same order as one group at a time).
constexpr int kL1Unroll = 4;
template <bool kVec>
__global__ __launch_bounds__(kL1Threads) void k_l1_partial(const float *image, const float *target, int64_t count,
                                                            float *grad, double *partial) {
    __shared__ double red[kL1Threads / kWave];
    const float inv = (float)(1.0 / (double)count);
    auto sgn = [inv](float r) { return r > 0.0f ? inv : (r < 0.0f ? -inv : 0.0f); };
    double s = 0.0;
    const int64_t tid = (int64_t)blockIdx.x * kL1Threads + threadIdx.x, stride = (int64_t)kL1Blocks * kL1Threads;
    int64_t i = tid;
    if (kVec) {
        const int64_t n4 = count / 4;
        const float4 *x4 = reinterpret_cast<const float4 *>(image), *y4 = reinterpret_cast<const float4 *>(target);
        float4 *g4 = reinterpret_cast<float4 *>(grad);
        int64_t q = tid;
        for (; q + (kL1Unroll - 1) * stride < n4; q += kL1Unroll * stride) {
            float4 x[kL1Unroll], y[kL1Unroll];
#pragma unroll
            for (int u = 0; u < kL1Unroll; ++u) {
                x[u] = x4[q + u * stride];
                y[u] = y4[q + u * stride];
            }
#pragma unroll
            for (int u = 0; u < kL1Unroll; ++u) {
                const float r0 = x[u].x - y[u].x, r1 = x[u].y - y[u].y, r2 = x[u].z - y[u].z, r3 = x[u].w - y[u].w;
                s += (double)fabsf(r0) + (double)fabsf(r1) + (double)fabsf(r2) + (double)fabsf(r3);
                if (grad) g4[q + u * stride] = make_float4(sgn(r0), sgn(r1), sgn(r2), sgn(r3));
            }
        }
        for (; q < n4; q += stride) {
            const float4 x = x4[q], y = y4[q];
            const float r0 = x.x - y.x, r1 = x.y - y.y, r2 = x.z - y.z, r3 = x.w - y.w;
            s += (double)fabsf(r0) + (double)fabsf(r1) + (double)fabsf(r2) + (double)fabsf(r3);
            if (grad) g4[q] = make_float4(sgn(r0), sgn(r1), sgn(r2), sgn(r3));
        }
        i = 4 * n4 + tid;
    }
    for (; i < count; i += stride) {
        const float r = image[i] - target[i];
        s += (double)fabsf(r);
        if (grad) grad[i] = sgn(r);
    }
    s = wave_sum(s);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kL1Threads / kWave; ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
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
// Photometric loss with the SSIM term, two kernels over 116 x 16 tiles.  The
// gradient at pixel p gathers the windows centred at q with |q - p| <= 5 (the
// window is symmetric); with S's partials A = dS/dmu_x, B = dS/ds_xx and
// C = dS/ds_xy at q it is
//   sum_q w(p - q) [A + 2 B (x_p - mu_x) + C (y_p - mu_y)]
//   = (G*D)(p) + 2 x_p (G*B)(p) + y_p (G*C)(p),   D = A - 2 B mu_x - C mu_y,
// (G* a window sum), so the first kernel writes the planes D, B, C at every
// pixel together with the per-tile sums of S and |x - y|, and the second
// filters them.  Both run one separable 11-tap pattern: the tile's inputs
// with a 5-pixel halo in LDS, a vertical pass (a thread per input column and
// 8 output rows, accumulating in registers), then a horizontal pass (a thread
// per row and 8 output columns) over the vertical sums, which reuse the LDS.
constexpr int kSsimR = 5;                      // window radius
constexpr int kTaps = 2 * kSsimR + 1;          // 11
constexpr int kSsimTW = 116;                   // output columns per tile
constexpr int kSsimTH = 16;                    // output rows per tile
constexpr int kSsimIW = kSsimTW + 2 * kSsimR;  // 126 input columns
constexpr int kSsimIH = kSsimTH + 2 * kSsimR;  // 26 input rows
constexpr int kRun = 8;                        // outputs per thread in each pass
constexpr int kGroups = (kSsimTW + kRun - 1) / kRun;      // 15 column groups
constexpr int kVPitch = kRun * (kGroups - 1) + kRun + kTaps - 1 + 1;  // 131 > the last group's reads
constexpr int kSsimThreads = 256;
constexpr int kPass1Items = kSsimIW * (kSsimTH / kRun);  // 252
constexpr int kPass2Items = kSsimTH * kGroups;            // 240
static_assert(kPass1Items <= kSsimThreads && kPass2Items <= kSsimThreads, "one item per thread");
static_assert(kSsimTH % kRun == 0, "whole runs of rows");
constexpr float kC1 = 0.01f * 0.01f, kC2 = 0.03f * 0.03f;

struct SsimArgs {
    const float *x, *y;
    const float *mask;  // [H][W] loss weights (null: all 1)
    float *planes;    // [3][channels][H][W]: D, B, C, weighted by the mask (null: loss only)
    float *grad;      // may be null
    double *partial;  // [tiles][3]: sums of m S, m |x - y| and m over the tile
    float *scale;     // 1 / (C sum m), written by the final reduction for the gradient
    int64_t plane_stride;  // channels * H * W
    int width, height, tiles_x, tiles_y, tiles, per_xcd;
    float w1[kTaps];  // normalised 1D Gaussian, sigma 1.5
    float lambda;
};

// Tile of this workgroup.  Consecutive workgroups go to the 8 XCDs in turn,
// so tile = (b mod 8) * per_xcd + b / 8 hands each XCD a contiguous run of
// tiles, ordered down the columns of tiles: a tile and its lower neighbour,
// whose input rows overlap, are read through the same L2.
__device__ inline int ssim_tile(const SsimArgs &a, int &c, int &tx0, int &ty0) {
    const int b = blockIdx.x;
    const int t = (b & 7) * a.per_xcd + (b >> 3);
    if (t >= a.tiles) return -1;
    const int rest = t / a.tiles_y;
    ty0 = (t - rest * a.tiles_y) * kSsimTH;
    c = rest / a.tiles_x;
    tx0 = (rest - c * a.tiles_x) * kSsimTW;
    return t;
}

// Inputs of the tile with their halo, zero outside the image.  Every load
// is issued before the first LDS store, so a workgroup waits for one round
// trip to HBM rather than one per row of threads.
constexpr int kHaloElems = kSsimIH * kSsimIW;
constexpr int kHaloIters = (kHaloElems + kSsimThreads - 1) / kSsimThreads;  // 13
template <int NIn>
__device__ inline void load_halo(float *lds, const float *const (&src)[NIn], int64_t plane_off, int tx0, int ty0,
                                 int width, int height) {
    float v[kHaloIters][NIn];
#pragma unroll
    for (int i = 0; i < kHaloIters; ++i) {
        const int k = threadIdx.x + i * kSsimThreads;
        const int r = k / kSsimIW, q = k - r * kSsimIW;
        const int gy = ty0 - kSsimR + r, gx = tx0 - kSsimR + q;
        const bool inside = k < kHaloElems && gy >= 0 && gy < height && gx >= 0 && gx < width;
        const int64_t off = plane_off + (int64_t)gy * width + gx;
#pragma unroll
        for (int p = 0; p < NIn; ++p) v[i][p] = inside ? src[p][off] : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < kHaloIters; ++i) {
        const int k = threadIdx.x + i * kSsimThreads;
        if (k < kHaloElems) {
#pragma unroll
            for (int p = 0; p < NIn; ++p) lds[p * kHaloElems + k] = v[i][p];
        }
    }
}

// Accumulate one input row (values v) into the kRun outputs it reaches: the
// t-th row of a run feeds output j with tap t - j.
template <int NV>
__device__ __forceinline__ void add_row(float (&acc)[kRun][NV], const float (&v)[NV], int t, const float *w) {
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
        const int tap = t - j;
        if (tap >= 0 && tap < kTaps) {
#pragma unroll
            for (int f = 0; f < NV; ++f) acc[j][f] = __builtin_fmaf(w[tap], v[f], acc[j][f]);
        }
    }
}

// Vertical sums -> LDS [NV][kSsimTH][kVPitch] (over the inputs, after a
// barrier), then the horizontal pass of this thread's item into m.
template <int NV>
__device__ inline void store_vertical(float *lds, const float (&acc)[kRun][NV], int k) {
    if (k >= kPass1Items) return;
    const int h = k / kSsimIW, q = k - h * kSsimIW;
#pragma unroll
    for (int j = 0; j < kRun; ++j)
#pragma unroll
        for (int f = 0; f < NV; ++f) lds[(f * kSsimTH + h * kRun + j) * kVPitch + q] = acc[j][f];
}

template <int NV>
__device__ inline void horizontal(const float *lds, int r, int g, const float *w, float (&m)[kRun][NV]) {
#pragma unroll
    for (int j = 0; j < kRun; ++j)
#pragma unroll
        for (int f = 0; f < NV; ++f) m[j][f] = 0.0f;
#pragma unroll
    for (int t = 0; t < kRun + kTaps - 1; ++t) {
        float v[NV];
#pragma unroll
        for (int f = 0; f < NV; ++f) v[f] = lds[(f * kSsimTH + r) * kVPitch + g * kRun + t];
        add_row<NV>(m, v, t, w);
    }
}

constexpr int kLdsStats = 5 * kSsimTH * kVPitch > 2 * kSsimIH * kSsimIW ? 5 * kSsimTH * kVPitch : 2 * kSsimIH * kSsimIW;
constexpr int kLdsGrad = 3 * kSsimTH * kVPitch > 3 * kSsimIH * kSsimIW ? 3 * kSsimTH * kVPitch : 3 * kSsimIH * kSsimIW;

// Window statistics, S, the planes D, B, C (weighted by the loss mask m at
// the window centre) and the tile's sums of m S, m |x - y| and m.
__global__ __launch_bounds__(kSsimThreads) void k_ssim_stats(SsimArgs a) {
    __shared__ float lds[kLdsStats];
    __shared__ double red[3][kSsimThreads / 64];
    int c, tx0, ty0;
    const int tile = ssim_tile(a, c, tx0, ty0);
    if (tile < 0) return;
    const int64_t plane = (int64_t)a.width * a.height;
    const float *const src[2] = {a.x, a.y};
    load_halo<2>(lds, src, c * plane, tx0, ty0, a.width, a.height);
    __syncthreads();
    const int k = threadIdx.x;
    // vertical pass over x, y, x^2, y^2, xy; |x - y| at the tile's own pixels
    float acc[kRun][5] = {};
    double l1_sum = 0.0;
    if (k < kPass1Items) {
        const int h = k / kSsimIW, q = k - h * kSsimIW;
        const int gx = tx0 - kSsimR + q;
        const bool own_col = q >= kSsimR && q < kSsimR + kSsimTW && gx < a.width;
        // loss weights of this column's own pixels (zero outside the image)
        float mw[kRun];
#pragma unroll
        for (int j = 0; j < kRun; ++j) {
            const int gy = ty0 + h * kRun + j;
            mw[j] = !a.mask ? 1.0f : (own_col && gy < a.height ? a.mask[(int64_t)gy * a.width + gx] : 0.0f);
        }
        float l1 = 0.0f;
#pragma unroll
        for (int t = 0; t < kRun + kTaps - 1; ++t) {
            const int row = h * kRun + t;
            const float xv = lds[row * kSsimIW + q], yv = lds[(kSsimIH + row) * kSsimIW + q];
            const float v[5] = {xv, yv, xv * xv, yv * yv, xv * yv};
            add_row<5>(acc, v, t, a.w1);
            if (t >= kSsimR && t < kSsimR + kRun) l1 = __builtin_fmaf(mw[t - kSsimR], fabsf(xv - yv), l1);
        }
        if (own_col) l1_sum = (double)l1;
    }
    __syncthreads();
    store_vertical<5>(lds, acc, k);
    __syncthreads();
    double s_sum = 0.0, m_sum = 0.0;
    if (k < kPass2Items) {
        const int r = k % kSsimTH, g = k / kSsimTH;
        float m[kRun][5];
        horizontal<5>(lds, r, g, a.w1, m);
        const int gy = ty0 + r;
#pragma unroll
        for (int j = 0; j < kRun; ++j) {
            const int col = g * kRun + j, gx = tx0 + col;
            if (col >= kSsimTW || gx >= a.width || gy >= a.height) continue;
            const float wq = a.mask ? a.mask[(int64_t)gy * a.width + gx] : 1.0f;
            m_sum += (double)wq;
            const float mx = m[j][0], my = m[j][1];
            const float vxx = m[j][2] - mx * mx, vyy = m[j][3] - my * my, vxy = m[j][4] - mx * my;
            const float n1 = 2.0f * mx * my + kC1, n2 = 2.0f * vxy + kC2;
            const float d1 = mx * mx + my * my + kC1, d2 = vxx + vyy + kC2;
            const float inv = 1.0f / (d1 * d2);
            const float S = n1 * n2 * inv;
            s_sum += (double)(wq * S);
            if (a.planes) {
                const float A = 2.0f * my * n2 * inv - S * 2.0f * mx / d1;  // dS/dmu_x
                const float B = -S / d2;                                    // dS/ds_xx
                const float C = 2.0f * n1 * inv;                            // dS/ds_xy
                const int64_t o = c * plane + (int64_t)gy * a.width + gx;
                a.planes[o] = wq * (A - 2.0f * B * mx - C * my);
                a.planes[a.plane_stride + o] = wq * B;
                a.planes[2 * a.plane_stride + o] = wq * C;
            }
        }
    }
    s_sum = wave_sum(s_sum);
    l1_sum = wave_sum(l1_sum);
    m_sum = wave_sum(m_sum);
    if ((k & 63) == 0) {
        red[0][k >> 6] = s_sum;
        red[1][k >> 6] = l1_sum;
        red[2][k >> 6] = m_sum;
    }
    __syncthreads();
    if (k == 0) {
        double s = 0.0, l = 0.0, mm = 0.0;
        for (int w = 0; w < kSsimThreads / 64; ++w) {
            s += red[0][w];
            l += red[1][w];
            mm += red[2][w];
        }
        a.partial[3 * tile] = s;
        a.partial[3 * tile + 1] = l;
        a.partial[3 * tile + 2] = mm;
    }
}

// dL/dx = [(1 - lambda) m sign(x - y) - lambda (G*D + 2 x G*B + y G*C)] / N
// with N = C sum m from the final reduction (the planes carry m already).
__global__ __launch_bounds__(kSsimThreads) void k_ssim_grad(SsimArgs a) {
    __shared__ float lds[kLdsGrad];
    int c, tx0, ty0;
    if (ssim_tile(a, c, tx0, ty0) < 0) return;
    const int64_t plane = (int64_t)a.width * a.height;
    const int k = threadIdx.x;
    // x, y at this thread's outputs, fetched while the passes run
    const int r = k % kSsimTH, g = k / kSsimTH;
    const int gy = ty0 + r;
    float xv[kRun], yv[kRun], mv[kRun];
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
        const int col = g * kRun + j, gx = tx0 + col;
        const bool own = k < kPass2Items && col < kSsimTW && gx < a.width && gy < a.height;
        const int64_t o = c * plane + (int64_t)gy * a.width + gx;
        xv[j] = own ? a.x[o] : 0.0f;
        yv[j] = own ? a.y[o] : 0.0f;
        mv[j] = !a.mask ? 1.0f : (own ? a.mask[(int64_t)gy * a.width + gx] : 0.0f);
    }
    const float *const src[3] = {a.planes, a.planes + a.plane_stride, a.planes + 2 * a.plane_stride};
    load_halo<3>(lds, src, c * plane, tx0, ty0, a.width, a.height);
    __syncthreads();
    float acc[kRun][3] = {};
    if (k < kPass1Items) {
        const int h = k / kSsimIW, q = k - h * kSsimIW;
#pragma unroll
        for (int t = 0; t < kRun + kTaps - 1; ++t) {
            const int row = h * kRun + t;
            const float v[3] = {lds[row * kSsimIW + q], lds[(kSsimIH + row) * kSsimIW + q],
                                lds[(2 * kSsimIH + row) * kSsimIW + q]};
            add_row<3>(acc, v, t, a.w1);
        }
    }
    __syncthreads();
    store_vertical<3>(lds, acc, k);
    __syncthreads();
    if (k >= kPass2Items || gy >= a.height) return;
    float m[kRun][3];
    horizontal<3>(lds, r, g, a.w1, m);
    const float l1w = 1.0f - a.lambda, inv_n = *a.scale;
#pragma unroll
    for (int j = 0; j < kRun; ++j) {
        const int col = g * kRun + j, gx = tx0 + col;
        if (col >= kSsimTW || gx >= a.width) continue;
        const int64_t o = c * plane + (int64_t)gy * a.width + gx;
        const float dS = m[j][0] + 2.0f * xv[j] * m[j][1] + yv[j] * m[j][2];
        const float d = xv[j] - yv[j];
        const float sgn = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
        a.grad[o] = inv_n * (l1w * mv[j] * sgn - a.lambda * dS);
    }
}

// loss = (1 - lambda) sum m|x - y| / N + lambda (1 - sum m S / N),
// N = sum over the tiles of sum m (C sum m over the pixels), in a fixed
// order; 1 / N goes to *scale for the gradient.
__global__ __launch_bounds__(256) void k_ssim_final(const double *partial, int64_t blocks, double lambda,
                                                    float *loss, float *scale) {
    __shared__ double red[3][256];
    double s = 0.0, l = 0.0, mm = 0.0;
    for (int64_t k = threadIdx.x; k < blocks; k += 256) {
        s += partial[3 * k];
        l += partial[3 * k + 1];
        mm += partial[3 * k + 2];
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = l;
    red[2][threadIdx.x] = mm;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
            red[2][threadIdx.x] += red[2][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n = red[2][0];
        *loss = (float)((1.0 - lambda) * red[1][0] / n + lambda * (1.0 - red[0][0] / n));
        *scale = (float)(1.0 / n);
    }
}

}  // namespace

static int64_t ssim_tiles(int channels, int height, int width) {
    return (int64_t)((width + kSsimTW - 1) / kSsimTW) * ((height + kSsimTH - 1) / kSsimTH) * channels;
}

// Scratch: per-tile partial sums (3 doubles per tile and channel), the
// gradient scale (one float in its own 256 bytes), then with a gradient the
// three filtered planes.
static size_t ssim_partial_bytes(int channels, int height, int width) {
    return ((size_t)ssim_tiles(channels, height, width) * 3 * sizeof(double) + 255) & ~(size_t)255;
}

size_t ssim_scratch_bytes(int channels, int height, int width, bool with_grad) {
    return ssim_partial_bytes(channels, height, width) + 256 +
           (with_grad ? (size_t)3 * channels * height * width * sizeof(float) : 0);
}

hipError_t launch_photometric(const float *image, const float *target, const float *mask, int channels, int height,
                              int width, float lambda, float *grad, float *loss, void *scratch, hipStream_t st) {
    SsimArgs a{};
    a.x = image;
    a.y = target;
    a.mask = mask;
    a.grad = grad;
    a.partial = static_cast<double *>(scratch);
    const size_t partial = ssim_partial_bytes(channels, height, width);
    a.scale = reinterpret_cast<float *>(static_cast<char *>(scratch) + partial);
    a.planes = grad ? reinterpret_cast<float *>(static_cast<char *>(scratch) + partial + 256) : nullptr;
    a.width = width;
    a.height = height;
    a.tiles_x = (width + kSsimTW - 1) / kSsimTW;
    a.tiles_y = (height + kSsimTH - 1) / kSsimTH;
    a.tiles = (int)ssim_tiles(channels, height, width);
    a.per_xcd = (a.tiles + 7) / 8;
    a.plane_stride = (int64_t)channels * height * width;
    double g[kTaps], sum = 0.0;
    for (int t = 0; t < kTaps; ++t) {
        const double d = t - kSsimR;
        g[t] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        sum += g[t];
    }
    for (int t = 0; t < kTaps; ++t) a.w1[t] = (float)(g[t] / sum);
    a.lambda = lambda;
    const dim3 grid((unsigned)(8 * a.per_xcd));
    hipLaunchKernelGGL(k_ssim_stats, grid, dim3(kSsimThreads), 0, st, a);
    hipLaunchKernelGGL(k_ssim_final, dim3(1), dim3(256), 0, st, a.partial, (int64_t)a.tiles, (double)lambda, loss,
                       a.scale);
    if (grad) hipLaunchKernelGGL(k_ssim_grad, grid, dim3(kSsimThreads), 0, st, a);
    return hipGetLastError();
}

size_t l1_scratch_bytes() { return kL1Blocks * sizeof(double); }

hipError_t launch_l1(const float *image, const float *target, int64_t count, float *grad, float *loss, void *scratch,
                     hipStream_t st) {
    double *partial = static_cast<double *>(scratch);
    auto aligned = [](const void *q) { return (reinterpret_cast<uintptr_t>(q) & 15u) == 0; };
    if (aligned(image) && aligned(target) && (!grad || aligned(grad)))
        hipLaunchKernelGGL(k_l1_partial<true>, dim3(kL1Blocks), dim3(kL1Threads), 0, st, image, target, count, grad,
                           partial);
    else
        hipLaunchKernelGGL(k_l1_partial<false>, dim3(kL1Blocks), dim3(kL1Threads), 0, st, image, target, count, grad,
                           partial);
    hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(kL1Threads), 0, st, partial, count, loss);
    return hipGetLastError();
}

}  // namespace omnigs
