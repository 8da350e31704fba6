// optim.hip -- the optimisation around the rasterizer (Sec. 4, Alg. 1): Adam
// on the raw parameters, densification statistics, densify / prune, opacity
// reset.  All HBM-bound elementwise or per-Gaussian passes.
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace omnigs {
namespace {

constexpr int kThreads = 256;

__device__ inline float sigmoidf_(float x) { return 1.0f / (1.0f + expf(-x)); }

// One Adam step of one element (x: parameter, g: gradient w.r.t. the
// activated value for log-scales and logits).
struct AdamOut {
    float x, m, v, act;
};
template <int kSeg>
__device__ __forceinline__ AdamOut adam_one(float x, float g, float m, float v, float lr, const AdamArgs &a) {
    if (kSeg == kSegLogScales) g *= expf(x);  // dS/dlog S = S
    if (kSeg == kSegLogits) {
        const float o = sigmoidf_(x);
        g *= o * (1.0f - o);  // do/dlogit
    }
    AdamOut r;
    r.m = a.beta1 * m + (1.0f - a.beta1) * g;
    r.v = a.beta2 * v + (1.0f - a.beta2) * (g * g);
    r.x = x - lr * a.inv_bc1 * r.m / (sqrtf(r.v) * a.inv_sqrt_bc2 + a.eps);
    r.act = kSeg == kSegLogScales ? expf(r.x) : (kSeg == kSegLogits ? sigmoidf_(r.x) : 0.0f);
    return r;
}

// One Adam step over one parameter array (blockIdx.y selects it): each
// thread takes four consecutive elements, as float4 when the arrays are
// 16-byte aligned.
template <int kSeg>
__device__ inline void adam_segment(const OptimArrays &P, const OptimArrays &G, const OptimArrays &M1,
                                    const OptimArrays &M2, const AdamArgs &a, float *act) {
    const int64_t len = (kSeg + 1 < kSegments ? a.begin[kSeg + 1] : a.total) - a.begin[kSeg];
    float *p = P.ptr[kSeg], *m = M1.ptr[kSeg], *v = M2.ptr[kSeg];
    const float *g = G.ptr[kSeg];
    const float lr = a.lr[kSeg];
    const bool vec = ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v) |
                       reinterpret_cast<uintptr_t>(g) | (act ? reinterpret_cast<uintptr_t>(act) : 0)) & 15u) == 0;
    const int64_t stride = (int64_t)gridDim.x * kThreads * 4;
    for (int64_t i0 = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * 4; i0 < len; i0 += stride) {
        if (vec && i0 + 4 <= len) {
            const float4 x4 = *reinterpret_cast<const float4 *>(p + i0), g4 = *reinterpret_cast<const float4 *>(g + i0);
            const float4 m4 = *reinterpret_cast<const float4 *>(m + i0), v4 = *reinterpret_cast<const float4 *>(v + i0);
            const float xs[4] = {x4.x, x4.y, x4.z, x4.w}, gs[4] = {g4.x, g4.y, g4.z, g4.w};
            const float ms[4] = {m4.x, m4.y, m4.z, m4.w}, vs[4] = {v4.x, v4.y, v4.z, v4.w};
            // column of i0 within its Gaussian's SH block (sh_stride >= 3, so
            // one wrap covers the next three)
            const int64_t c0 = kSeg == kSegSh ? i0 % a.sh_stride : 0;
            AdamOut r[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                float lk = lr;
                if (kSeg == kSegSh) {
                    int64_t c = c0 + k;
                    if (c >= a.sh_stride) c -= a.sh_stride;
                    if (c >= 3) lk = a.lr_sh_rest;  // SH degrees >= 1
                }
                r[k] = adam_one<kSeg>(xs[k], gs[k], ms[k], vs[k], lk, a);
            }
            *reinterpret_cast<float4 *>(p + i0) = make_float4(r[0].x, r[1].x, r[2].x, r[3].x);
            *reinterpret_cast<float4 *>(m + i0) = make_float4(r[0].m, r[1].m, r[2].m, r[3].m);
            *reinterpret_cast<float4 *>(v + i0) = make_float4(r[0].v, r[1].v, r[2].v, r[3].v);
            if ((kSeg == kSegLogScales || kSeg == kSegLogits) && act)
                *reinterpret_cast<float4 *>(act + i0) = make_float4(r[0].act, r[1].act, r[2].act, r[3].act);
        } else {
            for (int64_t i = i0; i < i0 + 4 && i < len; ++i) {
                float lk = lr;
                if (kSeg == kSegSh && (i % a.sh_stride) >= 3) lk = a.lr_sh_rest;
                const AdamOut r = adam_one<kSeg>(p[i], g[i], m[i], v[i], lk, a);
                p[i] = r.x;
                m[i] = r.m;
                v[i] = r.v;
                if ((kSeg == kSegLogScales || kSeg == kSegLogits) && act) act[i] = r.act;
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_adam(OptimArrays P, OptimArrays G, OptimArrays M1, OptimArrays M2,
                                                   AdamArgs a, float *act_scales, float *act_opacities,
                                                   const int32_t *skip) {
    if (skip && *skip) return;
    switch (blockIdx.y) {
        case kSegMeans: adam_segment<kSegMeans>(P, G, M1, M2, a, nullptr); break;
        case kSegLogScales: adam_segment<kSegLogScales>(P, G, M1, M2, a, act_scales); break;
        case kSegQuats: adam_segment<kSegQuats>(P, G, M1, M2, a, nullptr); break;
        case kSegLogits: adam_segment<kSegLogits>(P, G, M1, M2, a, act_opacities); break;
        default: adam_segment<kSegSh>(P, G, M1, M2, a, nullptr); break;
    }
}

__global__ __launch_bounds__(kThreads) void k_stats(const uint32_t *n_tiles, const float *radii, const float *dscreen,
                                                    int64_t n, float *accum, float *denom, float *max_radius,
                                                    const int32_t *skip) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n || (skip && *skip) || n_tiles[i] == 0) return;
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
                       const AdamArgs &a, float *act_scales, float *act_opacities, const int32_t *skip,
                       hipStream_t st) {
    if (a.total == 0) return hipSuccess;
    // blockIdx.y: the parameter array; x: enough blocks for the largest (SH)
    int64_t longest = 0;
    for (int k = 0; k < kSegments; ++k)
        longest = std::max<int64_t>(longest, (k + 1 < kSegments ? a.begin[k + 1] : a.total) - a.begin[k]);
    const unsigned grid = (unsigned)std::min<int64_t>((longest + 4 * kThreads - 1) / (4 * kThreads), 256 * 32);
    hipLaunchKernelGGL(k_adam, dim3(grid, kSegments), dim3(kThreads), 0, st, P, G, M1, M2, a, act_scales,
                       act_opacities, skip);
    return hipGetLastError();
}

hipError_t launch_stats(const uint32_t *n_tiles, const float *radii, const float *dscreen, int64_t n, float *accum,
                        float *denom, float *max_radius, const int32_t *skip, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_stats, dim3(blocks(n)), dim3(kThreads), 0, st, n_tiles, radii, dscreen, n, accum, denom,
                       max_radius, skip);
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
