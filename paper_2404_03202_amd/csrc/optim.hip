// optim.hip -- the optimisation around the rasterizer (Sec. 4, Alg. 1): Adam
// on the raw parameters, densification statistics, densify / prune, opacity
// reset.  All HBM-bound elementwise or per-Gaussian passes.
#include "internal.h"

#include <cmath>

namespace omnigs {
namespace {

constexpr int kThreads = 256;

__device__ inline float sigmoidf_(float x) { return 1.0f / (1.0f + expf(-x)); }

// One Adam step over the concatenation of the parameter arrays (means,
// log_scales, quats, logits, sh); segment boundaries in elements.
__global__ __launch_bounds__(kThreads) void k_adam(OptimArrays P, OptimArrays G, OptimArrays M1, OptimArrays M2,
                                                   AdamArgs a, float *act_scales, float *act_opacities) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < a.total; e += stride) {
        int seg = 0;
#pragma unroll
        for (int k = 1; k < kSegments; ++k) seg += e >= a.begin[k] ? 1 : 0;
        const int64_t i = e - a.begin[seg];
        float *p = P.ptr[seg] + i, *m = M1.ptr[seg] + i, *v = M2.ptr[seg] + i;
        float g = G.ptr[seg][i];
        const float x = *p;
        float lr = a.lr[seg];
        if (seg == kSegLogScales) g *= expf(x);                    // dS/dlog S = S
        if (seg == kSegLogits) {
            const float o = sigmoidf_(x);
            g *= o * (1.0f - o);                                    // do/dlogit
        }
        if (seg == kSegSh && (i % a.sh_stride) >= 3) lr = a.lr_sh_rest;  // SH degrees >= 1
        const float mn = a.beta1 * *m + (1.0f - a.beta1) * g;
        const float vn = a.beta2 * *v + (1.0f - a.beta2) * (g * g);
        const float xn = x - lr * a.inv_bc1 * mn / (sqrtf(vn) * a.inv_sqrt_bc2 + a.eps);
        *m = mn;
        *v = vn;
        *p = xn;
        if (seg == kSegLogScales && act_scales) act_scales[i] = expf(xn);
        if (seg == kSegLogits && act_opacities) act_opacities[i] = sigmoidf_(xn);
    }
}

__global__ __launch_bounds__(kThreads) void k_stats(const uint32_t *n_tiles, const float *radii, const float *dscreen,
                                                    int64_t n, float *accum, float *denom, float *max_radius) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n || n_tiles[i] == 0) return;
    const float gx = dscreen[2 * i], gy = dscreen[2 * i + 1];
    accum[i] += sqrtf(gx * gx + gy * gy);
    denom[i] += 1.0f;
    max_radius[i] = fmaxf(max_radius[i], radii[i]);
}

// Keep flags in four blocks of n: originals, clones, first children,
// second children (the same flag twice).
__global__ __launch_bounds__(kThreads) void k_dens_flags(OptimArrays P, const float *accum, const float *denom,
                                                         const float *max_radius, int64_t n, DensifyArgs d,
                                                         uint32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const float *ls = P.ptr[kSegLogScales] + 3 * i;
    const float lsmax = fmaxf(fmaxf(ls[0], ls[1]), ls[2]);
    const float child_lsmax = fmaxf(fmaxf(ls[0] - d.log_shrink, ls[1] - d.log_shrink), ls[2] - d.log_shrink);
    const float dn = denom[i];
    const float gm = dn > 0.0f ? accum[i] / dn : 0.0f;  // correctly rounded float division
    const bool hot = gm >= d.tau;
    const bool small = lsmax <= d.log_clone;
    const bool clone = hot && small, split = hot && !small;
    const bool low = P.ptr[kSegLogits][i] < d.logit_min;
    const bool prune_big = d.screen_on && (max_radius[i] > d.max_screen || lsmax > d.log_big);
    const bool clone_big = d.screen_on && (0.0f > d.max_screen || lsmax > d.log_big);
    const bool child_big = d.screen_on && (0.0f > d.max_screen || child_lsmax > d.log_big);
    flags[i] = (!split && !low && !prune_big) ? 1u : 0u;
    flags[n + i] = (clone && !low && !clone_big) ? 1u : 0u;
    const uint32_t kid = (split && !low && !child_big) ? 1u : 0u;
    flags[2 * n + i] = kid;
    flags[3 * n + i] = kid;
}

__device__ inline void copy_params(const OptimArrays &S, int64_t i, const OptimArrays &D, int64_t j, int sh_floats) {
    for (int k = 0; k < 3; ++k) D.ptr[kSegMeans][3 * j + k] = S.ptr[kSegMeans][3 * i + k];
    for (int k = 0; k < 3; ++k) D.ptr[kSegLogScales][3 * j + k] = S.ptr[kSegLogScales][3 * i + k];
    for (int k = 0; k < 4; ++k) D.ptr[kSegQuats][4 * j + k] = S.ptr[kSegQuats][4 * i + k];
    D.ptr[kSegLogits][j] = S.ptr[kSegLogits][i];
    for (int k = 0; k < sh_floats; ++k) D.ptr[kSegSh][(int64_t)sh_floats * j + k] = S.ptr[kSegSh][(int64_t)sh_floats * i + k];
}

__device__ inline void zero_params(const OptimArrays &D, int64_t j, int sh_floats) {
    for (int k = 0; k < 3; ++k) D.ptr[kSegMeans][3 * j + k] = 0.0f;
    for (int k = 0; k < 3; ++k) D.ptr[kSegLogScales][3 * j + k] = 0.0f;
    for (int k = 0; k < 4; ++k) D.ptr[kSegQuats][4 * j + k] = 0.0f;
    D.ptr[kSegLogits][j] = 0.0f;
    for (int k = 0; k < sh_floats; ++k) D.ptr[kSegSh][(int64_t)sh_floats * j + k] = 0.0f;
}

__global__ __launch_bounds__(kThreads) void k_dens_scatter(OptimArrays P, OptimArrays M1, OptimArrays M2,
                                                           const uint32_t *flags, const uint32_t *pos, const float *noise,
                                                           int64_t n, int sh_floats, float log_shrink, OptimArrays PO,
                                                           OptimArrays M1O, OptimArrays M2O) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    if (flags[i]) {
        const int64_t j = pos[i];
        copy_params(P, i, PO, j, sh_floats);
        copy_params(M1, i, M1O, j, sh_floats);
        copy_params(M2, i, M2O, j, sh_floats);
    }
    if (flags[n + i]) {
        const int64_t j = pos[n + i];
        copy_params(P, i, PO, j, sh_floats);
        zero_params(M1O, j, sh_floats);
        zero_params(M2O, j, sh_floats);
    }
    if (!flags[2 * n + i]) return;
    // children: m + R(q) (S * z), S = exp(log_scales)
    const float *q = P.ptr[kSegQuats] + 4 * i;
    const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const float w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    const float R[9] = {1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y),
                        2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x),
                        2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)};
    const float *ls = P.ptr[kSegLogScales] + 3 * i;
    const float S[3] = {expf(ls[0]), expf(ls[1]), expf(ls[2])};
    for (int c = 0; c < 2; ++c) {
        const int64_t j = pos[(2 + c) * n + i];
        copy_params(P, i, PO, j, sh_floats);
        const float *zz = noise + 6 * i + 3 * c;
        for (int r = 0; r < 3; ++r)
            PO.ptr[kSegMeans][3 * j + r] = P.ptr[kSegMeans][3 * i + r] + R[3 * r] * (S[0] * zz[0]) +
                                           R[3 * r + 1] * (S[1] * zz[1]) + R[3 * r + 2] * (S[2] * zz[2]);
        for (int r = 0; r < 3; ++r) PO.ptr[kSegLogScales][3 * j + r] = ls[r] - log_shrink;
        zero_params(M1O, j, sh_floats);
        zero_params(M2O, j, sh_floats);
    }
}

__global__ __launch_bounds__(kThreads) void k_reset_opacity(float *logits, float *m1, float *m2, int64_t n, float lo) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    logits[i] = fminf(logits[i], lo);
    m1[i] = 0.0f;
    m2[i] = 0.0f;
}

unsigned blocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_adam(const OptimArrays &P, const OptimArrays &G, const OptimArrays &M1, const OptimArrays &M2,
                       const AdamArgs &a, float *act_scales, float *act_opacities, hipStream_t st) {
    if (a.total == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<int64_t>((a.total + kThreads - 1) / kThreads, 256 * 64);
    hipLaunchKernelGGL(k_adam, dim3(grid), dim3(kThreads), 0, st, P, G, M1, M2, a, act_scales, act_opacities);
    return hipGetLastError();
}

hipError_t launch_stats(const uint32_t *n_tiles, const float *radii, const float *dscreen, int64_t n, float *accum,
                        float *denom, float *max_radius, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_stats, dim3(blocks(n)), dim3(kThreads), 0, st, n_tiles, radii, dscreen, n, accum, denom,
                       max_radius);
    return hipGetLastError();
}

hipError_t launch_dens_flags(const OptimArrays &P, const float *accum, const float *denom, const float *max_radius,
                             int64_t n, const DensifyArgs &d, uint32_t *flags, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dens_flags, dim3(blocks(n)), dim3(kThreads), 0, st, P, accum, denom, max_radius, n, d, flags);
    return hipGetLastError();
}

hipError_t launch_dens_scatter(const OptimArrays &P, const OptimArrays &M1, const OptimArrays &M2,
                               const uint32_t *flags, const uint32_t *pos, const float *noise, int64_t n,
                               int sh_floats, float log_shrink, const OptimArrays &PO, const OptimArrays &M1O,
                               const OptimArrays &M2O, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_dens_scatter, dim3(blocks(n)), dim3(kThreads), 0, st, P, M1, M2, flags, pos, noise, n,
                       sh_floats, log_shrink, PO, M1O, M2O);
    return hipGetLastError();
}

hipError_t launch_reset_opacity(float *logits, float *m1, float *m2, int64_t n, float lo, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reset_opacity, dim3(blocks(n)), dim3(kThreads), 0, st, logits, m1, m2, n, lo);
    return hipGetLastError();
}

}  // namespace omnigs
