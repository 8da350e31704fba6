// blend.hip -- front-to-back alpha blending of the sorted tile lists (Eq. 6-8,
// Sec. 3.3) and its reverse-order backward (Sec. 3.4).
//
// One workgroup of 256 lanes (four wave64s) per 16x16 tile, one lane per
// pixel.  The workgroup stages the next 256 instances of its tile list in
// LDS (each lane gathers one 48-byte record), then every lane walks the
// staged batch.  Positions are made tile-relative when staged, from the
// record's hi/lo split, so per-pixel offsets keep full precision at any
// image width; the x offset is then wrapped to the shortest signed offset
// on the circle of circumference W (the longitude seam).
//
// alpha = min(alpha_max, o * exp(-1/2 d^T Q d)) is evaluated by one inline
// function in both kernels, with explicit FMAs, so that the backward re-walk
// takes exactly the forward's decisions (skip below alpha_min, stop before
// T < T_min) from the saved final T and contributor count.
//
// The backward reduces each instance's nine per-pixel gradient terms over
// the wave (DPP row sums plus two cross-row shuffles) and over the four
// waves (LDS), then issues one float atomic per field per (tile, instance).
#include "internal.h"

namespace omnigs {
namespace {

constexpr float kLog2e = 1.4426950408889634f;

struct BlendFrame {
    int width, height, tiles_x, tiles_y;
    uint32_t tile_base;
    float *image;
    float *final_T;
    int32_t *n_contrib;
    const float *dL;  // backward only
};

constexpr int kMaxFrames = 32;
struct FrameTable {
    int n;
    BlendFrame f[kMaxFrames];
};

__device__ inline int find_frame(const FrameTable &T, uint32_t tile) {
    int f = 0;
    for (int k = 1; k < T.n; ++k)
        if (tile >= T.f[k].tile_base) f = k;
    return f;
}

// Stage one instance in LDS: position relative to the tile origin, conic
// pre-scaled so that the exponent is evaluated in base 2:
//   p2 = c00 dx^2 + c01 dx dy + c11 dy^2 = log2(e) * (-1/2 d^T Q d).
__device__ inline void stage(const BlendRecord *rec, uint32_t gid, float X0, float Y0, float W, float *sx,
                             float *sy, float4 *sc, float4 *scol, int slot) {
    const float4 *p = reinterpret_cast<const float4 *>(rec + gid);
    const float4 a = p[0], b = p[1], c = p[2];
    float x = (a.x - X0) + a.y;  // px_hi - X0 is exact near the tile
    const float y = (a.z - Y0) + a.w;
    // bring the centre within half a turn of the tile's middle column
    const float half = 0.5f * W;
    if (x - 8.0f >= half) x -= W;
    if (x - 8.0f < -half) x += W;
    sx[slot] = x;
    sy[slot] = y;
    sc[slot] = make_float4(-0.5f * kLog2e * b.x, -kLog2e * b.y, -0.5f * kLog2e * b.z, b.w);
    scol[slot] = c;
}

// alpha of one staged instance at pixel centre (fx, fy) (tile-relative);
// returns the unclamped alpha, writes the clamped one and the pixel offset.
__device__ __forceinline__ float eval_alpha(float fx, float fy, float x, float y, float4 conic, float W, float half,
                                            float alpha_max, float &alpha, float &dx, float &dy, float &G) {
    float d = fx - x;
    d = (d >= half) ? d - W : d;
    d = (d < -half) ? d + W : d;
    dx = d;
    dy = fy - y;
    const float t = __builtin_fmaf(conic.y, dy, conic.x * dx);
    const float p2 = __builtin_fmaf(conic.z * dy, dy, dx * t);
    G = __builtin_amdgcn_exp2f(p2);
    const float araw = conic.w * G;
    alpha = araw < alpha_max ? araw : alpha_max;
    return araw;
}

template <bool kBatched>
__global__ __launch_bounds__(kBlendThreads) void k_blend_forward(FrameTable FT, const BlendRecord *rec,
                                                                  const uint32_t *inst_gauss, const uint2 *ranges,
                                                                  BlendSettings s) {
    __shared__ float sx[kBlendThreads], sy[kBlendThreads];
    __shared__ float4 sc[kBlendThreads], scol[kBlendThreads];
    const uint32_t tile = blockIdx.x;
    const int fi = kBatched ? find_frame(FT, tile) : 0;
    const BlendFrame &F = FT.f[fi];
    const uint32_t lt = tile - F.tile_base;
    const int tx = lt % F.tiles_x, ty = lt / F.tiles_x;
    const int lx = threadIdx.x % kTile, ly = threadIdx.x / kTile;
    const int x = tx * kTile + lx, y = ty * kTile + ly;
    const bool inside = y < F.height;
    const float W = (float)F.width, half = 0.5f * W;
    const float X0 = (float)(tx * kTile), Y0 = (float)(ty * kTile);
    const float fx = lx + 0.5f, fy = ly + 0.5f;
    const uint2 range = ranges[tile];
    const int count = (int)(range.y - range.x);
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    int last = 0;
    bool done = !inside;
    for (int base = 0; base < count; base += kBlendThreads) {
        if (__syncthreads_count(done) == kBlendThreads) break;
        const int k = base + threadIdx.x;
        if (k < count) stage(rec, inst_gauss[range.x + k], X0, Y0, W, sx, sy, sc, scol, threadIdx.x);
        __syncthreads();
        const int nb = min(kBlendThreads, count - base);
        for (int j = 0; !done && j < nb; ++j) {
            float alpha, dx, dy, G;
            eval_alpha(fx, fy, sx[j], sy[j], sc[j], W, half, s.alpha_max, alpha, dx, dy, G);
            if (alpha < s.alpha_min) continue;
            const float Tn = T * (1.0f - alpha);
            if (Tn < s.T_min) {
                done = true;
                break;
            }
            const float wgt = alpha * T;
            const float4 col = scol[j];
            C0 = __builtin_fmaf(col.x, wgt, C0);
            C1 = __builtin_fmaf(col.y, wgt, C1);
            C2 = __builtin_fmaf(col.z, wgt, C2);
            T = Tn;
            last = base + j + 1;
        }
    }
    if (inside) {
        const int64_t HW = (int64_t)F.width * F.height;
        const int64_t p = (int64_t)y * F.width + x;
        F.image[p] = __builtin_fmaf(T, s.bg[0], C0);
        F.image[HW + p] = __builtin_fmaf(T, s.bg[1], C1);
        F.image[2 * HW + p] = __builtin_fmaf(T, s.bg[2], C2);
        F.final_T[p] = T;
        F.n_contrib[p] = last;
    }
}

// Sum over the 64 lanes of the wave; every lane receives the total.
__device__ __forceinline__ float wave_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));  // xor 1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));  // xor 2
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x124, 0xF, 0xF, false)); // ror 4
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x128, 0xF, 0xF, false)); // ror 8
    v += __shfl_xor(v, 16, kWave);
    v += __shfl_xor(v, 32, kWave);
    return v;
}

template <bool kBatched>
__global__ __launch_bounds__(kBlendThreads) void k_blend_backward(FrameTable FT, const BlendRecord *rec,
                                                                   const uint32_t *inst_gauss, const uint2 *ranges,
                                                                   BlendSettings s, float *acc) {
    constexpr int kW = kBlendThreads / kWave;
    __shared__ float sx[kBlendThreads], sy[kBlendThreads];
    __shared__ float4 sc[kBlendThreads], scol[kBlendThreads];
    __shared__ uint32_t sgid[kBlendThreads];
    __shared__ float part[kBlendThreads][kW][kAcc];
    __shared__ int s_max_last;
    const uint32_t tile = blockIdx.x;
    const int fi = kBatched ? find_frame(FT, tile) : 0;
    const BlendFrame &F = FT.f[fi];
    const uint32_t lt = tile - F.tile_base;
    const int tx = lt % F.tiles_x, ty = lt / F.tiles_x;
    const int lx = threadIdx.x % kTile, ly = threadIdx.x / kTile;
    const int x = tx * kTile + lx, y = ty * kTile + ly;
    const bool inside = y < F.height;
    const float W = (float)F.width, half = 0.5f * W;
    const float X0 = (float)(tx * kTile), Y0 = (float)(ty * kTile);
    const float fx = lx + 0.5f, fy = ly + 0.5f;
    const uint2 range = ranges[tile];
    const int wave = threadIdx.x / kWave;
    float T = 1.0f, dL0 = 0.0f, dL1 = 0.0f, dL2 = 0.0f;
    int last = 0;
    if (inside) {
        const int64_t HW = (int64_t)F.width * F.height;
        const int64_t p = (int64_t)y * F.width + x;
        T = F.final_T[p];
        last = F.n_contrib[p];
        dL0 = F.dL[p];
        dL1 = F.dL[HW + p];
        dL2 = F.dL[2 * HW + p];
    }
    // dL . (colour blended behind the current instance + T_final bg)
    float dLS = T * (dL0 * s.bg[0] + dL1 * s.bg[1] + dL2 * s.bg[2]);
    if (threadIdx.x == 0) s_max_last = 0;
    __syncthreads();
    atomicMax(&s_max_last, last);
    __syncthreads();
    const int max_last = s_max_last;
    for (int hi = max_last; hi > 0; hi -= kBlendThreads) {
        const int lo = hi - kBlendThreads > 0 ? hi - kBlendThreads : 0;
        const int nb = hi - lo;
        __syncthreads();
        if (threadIdx.x < nb) {
            const int pos = hi - 1 - threadIdx.x;  // slot j holds list position hi-1-j
            const uint32_t g = inst_gauss[range.x + pos];
            sgid[threadIdx.x] = g;
            stage(rec, g, X0, Y0, W, sx, sy, sc, scol, threadIdx.x);
        }
        __syncthreads();
        for (int j = 0; j < nb; ++j) {
            const int pos = hi - 1 - j;
            float v[kAcc];
#pragma unroll
            for (int k = 0; k < kAcc; ++k) v[k] = 0.0f;
            bool any = false;
            if (pos < last) {
                float alpha, dx, dy, G;
                const float4 conic = sc[j];
                const float araw = eval_alpha(fx, fy, sx[j], sy[j], conic, W, half, s.alpha_max, alpha, dx, dy, G);
                if (alpha >= s.alpha_min) {
                    any = true;
                    const float one_m = 1.0f - alpha;
                    const float inv = 1.0f / one_m;
                    T = T * inv;  // transmittance in front of this instance
                    const float wgt = alpha * T;
                    const float4 col = scol[j];
                    const float dLc = dL0 * col.x + dL1 * col.y + dL2 * col.z;
                    const float dalpha = dLc * T - dLS * inv;
                    dLS = __builtin_fmaf(dLc, wgt, dLS);
                    v[6] = dL0 * wgt;
                    v[7] = dL1 * wgt;
                    v[8] = dL2 * wgt;
                    if (araw < s.alpha_max) {
                        const float gp = araw * dalpha;  // dL/d(-1/2 d^T Q d)
                        v[0] = dx * gp;
                        v[1] = dy * gp;
                        v[2] = dx * v[0];
                        v[3] = dx * v[1];
                        v[4] = dy * v[1];
                        v[5] = G * dalpha;
                    }
                }
            }
            const bool wave_any = __ballot(any) != 0ull;
            if (wave_any) {
#pragma unroll
                for (int k = 0; k < kAcc; ++k) v[k] = wave_sum(v[k]);
            }
            if (__lane_id() == 0) {
#pragma unroll
                for (int k = 0; k < kAcc; ++k) part[j][wave][k] = v[k];
            }
        }
        __syncthreads();
        // fold the four waves' partial sums; moments -> screen-space gradients
        for (int j = threadIdx.x; j < nb; j += kBlendThreads) {
            float m[kAcc];
#pragma unroll
            for (int k = 0; k < kAcc; ++k) m[k] = part[j][0][k] + part[j][1][k] + part[j][2][k] + part[j][3][k];
            // conic back to Q: q00 = -2 ln2 c00, q01 = -ln2 c01, q11 = -2 ln2 c11
            const float4 c = sc[j];
            const float q00 = -2.0f * c.x / kLog2e, q01 = -c.y / kLog2e, q11 = -2.0f * c.z / kLog2e;
            float out[kAcc];
            out[0] = q00 * m[0] + q01 * m[1];  // dL/dp_x
            out[1] = q01 * m[0] + q11 * m[1];  // dL/dp_y
            out[2] = -0.5f * m[2];             // dL/dq00
            out[3] = -m[3];                    // dL/dq01
            out[4] = -0.5f * m[4];             // dL/dq11
            out[5] = m[5];                     // dL/do
            out[6] = m[6];
            out[7] = m[7];
            out[8] = m[8];
            float *dst = acc + (int64_t)sgid[j] * kAcc;
#pragma unroll
            for (int k = 0; k < kAcc; ++k)
                if (out[k] != 0.0f) atomicAdd(dst + k, out[k]);
        }
    }
}

}  // namespace

hipError_t launch_blend_forward(const FrameGeom &f, const BlendRecord *rec, const uint32_t *inst_gauss,
                                const uint2 *ranges, const BlendSettings &s, float *image, float *final_T,
                                int32_t *n_contrib, hipStream_t st) {
    FrameTable T{};
    T.n = 1;
    T.f[0] = BlendFrame{f.width, f.height, f.tiles_x, f.tiles_y, f.tile_base, image, final_T, n_contrib, nullptr};
    const unsigned tiles = (unsigned)(f.tiles_x * f.tiles_y);
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_blend_forward<false>, dim3(tiles), dim3(kBlendThreads), 0, st, T, rec, inst_gauss,
                       ranges + f.tile_base, s);
    return hipGetLastError();
}

hipError_t launch_blend_backward(const FrameGeom &f, const BlendRecord *rec, const uint32_t *inst_gauss,
                                 const uint2 *ranges, const BlendSettings &s, const float *final_T,
                                 const int32_t *n_contrib, const float *dL_dimage, float *acc, hipStream_t st) {
    FrameTable T{};
    T.n = 1;
    T.f[0] = BlendFrame{f.width, f.height, f.tiles_x, f.tiles_y, f.tile_base, nullptr, const_cast<float *>(final_T),
                        const_cast<int32_t *>(n_contrib), dL_dimage};
    const unsigned tiles = (unsigned)(f.tiles_x * f.tiles_y);
    if (tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_blend_backward<false>, dim3(tiles), dim3(kBlendThreads), 0, st, T, rec, inst_gauss,
                       ranges + f.tile_base, s, acc);
    return hipGetLastError();
}

}  // namespace omnigs
