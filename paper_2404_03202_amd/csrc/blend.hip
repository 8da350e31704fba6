// blend.hip -- front-to-back alpha blending of the sorted tile lists (Eq. 6-8,
// Sec. 3.3) and its reverse-order backward (Sec. 3.4).
//
// One workgroup per 16x16 tile, of kW wave64s (1, 2 or 4; a template
// parameter, chosen separately for the two kernels).  The tile's four 8x8
// quadrants are split between the waves; each lane owns one pixel of each
// quadrant of its wave (4 / kW pixels).  More waves shorten the longest
// per-wave walk (a tile's list is split by quadrant); more pixels per lane
// amortise the backward's cross-lane reduction over more pixels.
//
// The workgroup stages the next kBatch = 64 kW instances of its tile list in
// LDS (each lane gathers one 48-byte record); positions are made
// tile-relative from the record's hi/lo split, so pixel offsets keep full
// precision at any width.  The x offset is the shortest signed offset on the
// circle of circumference W (the longitude seam of the ERP image; a pinhole
// image sets the period to infinity, so nothing wraps).  Pixels past the
// image's right or bottom edge (partial last tiles) never blend.
//
// An instance whose centre is a turn away for part of the tile's columns
// (seam split, below) is rare; a wave walks a batch with the per-column
// centre select only when its list holds one (a uniform branch between two
// instantiations of the walk).
//
// The lane that stages an instance also tests which quadrants its
// alpha >= alpha_min ellipse can reach (the exact minimum of the quadratic
// form over each quadrant's pixel-centre rectangle, with a safety margin).
// Each wave then compacts, in order, the staged instances that reach one of
// its quadrants and walks only those, skipping unreached quadrants with a
// uniform branch: a skipped instance holds no pixel of the quadrant whose
// alpha could pass alpha_min, so the image is unchanged.
//
// alpha = min(alpha_max, o * exp(-1/2 d^T Q d)) is evaluated per pixel by the
// same inline function in both kernels, with explicit FMAs (the library is
// built without FP contraction), and both use the same quadrant test, so the
// backward re-walk takes exactly the forward's decisions (skip below
// alpha_min, stop before T < T_min) from the saved final T and contributor
// count, whatever the wave layout of each kernel.
//
// Backward reduction: a wave reduce-scatters an instance's nine gradient
// terms across its lanes (gfx950 permlane swaps between wave halves and
// between rows, then DPP mirror and quad steps inside the rows, every
// exchange carrying two fields: no LDS traffic), and the nine lanes holding
// the sums add them into the instance's LDS slot in one instruction; after
// the batch, the lane that staged the instance converts the sums to
// screen-space gradients in place, and the workgroup
// adds them to global memory with float atomics (one per nonzero field per
// (tile, instance)), issued field-contiguous: consecutive lanes take
// consecutive fields of the same few Gaussians.
#include "internal.h"

#ifndef OMNIGS_FWD_WAVES
#define OMNIGS_FWD_WAVES 4
#endif
#ifndef OMNIGS_BWD_WAVES
#define OMNIGS_BWD_WAVES 2
#endif

namespace omnigs {
namespace {

constexpr float kLn2 = 0.69314718055994531f;
constexpr int kQuads = 4;  // 8x8 quadrants per tile
constexpr uint32_t kSplitBit = 1u << 31;  // staged quad mask: seam split inside the tile

struct BlendFrame {
    int width, height, tiles_x, tiles_y;
    uint32_t tile_base;
    float period;  // x wrap period: the width (ERP) or +infinity (pinhole)
    float *image;
    float *final_T;
    int32_t *n_contrib;
    int32_t *n_blended;  // forward only, may be null
    const float *dL;     // backward only
    float *depth;        // forward only: the depth image (with kAux)
    const float *dLD;    // backward only: dL/ddepth, may be null
    const float *dLA;    // backward only: dL/dalpha, may be null
    // per tile instance (indexed as the instance lists), the reach mask of its
    // quadrants: written by the forward for every instance it stages, read by
    // the backward in place of the quadrant tests (null: computed)
    uint8_t *quad;
};

struct FrameTable {
    int n;
    BlendFrame f[kMaxBatch];
};

__device__ inline int find_frame(const FrameTable &T, uint32_t tile) {
    int f = 0;
    for (int k = 1; k < T.n; ++k)
        if (tile >= T.f[k].tile_base) f = k;
    return f;
}

// Staged instances (LDS):
//   a = (u0a, v0, l00, l10), b = (l11, log2 o, r, g), c = (b, u0b, thr, depth),
//   quad = quadrant mask
// with L the record's scaled Cholesky factor of the conic:
// -(l00 dx + l10 dy)^2 - (l11 dy)^2 = log2(e) * (-1/2 d^T Q d).  The pixel at
// integer tile coordinates (i, j) has d = (i + 1/2 - x, j + 1/2 - y) with the
// centre x relative to the tile origin taken as xa for i < thr and as xb for
// i >= thr: thr lies past the tile (xb unused) except where the offsets of
// the tile's columns cross the seam (a centre near the antipode of the
// tile); there xb = xa + W and thr splits the columns.  So L^T d = (l00 i + l10 j + u0, l11 j +
// v0) with u0 = u0a or u0b, formed once per (tile, instance) in double
// precision: a pixel pays a compare, a select and three FMAs for L^T d.
// The quadrant mask sits in c.w (its bits) when no depth is staged (kAux
// false), else in quad[].  list[w] holds, for wave w, the staged slots that
// reach one of its quadrants, in order, as slot | (wave mask << 8).
template <int kW>
struct StageCore {
    static constexpr int kBatch = kWave * kW;
    float4 a[kBatch], b[kBatch], c[kBatch];
    uint16_t list[kW][kBatch];
};
template <int kW, bool kAux>
struct Stage : StageCore<kW> {
    uint32_t quad[StageCore<kW>::kBatch];
    __device__ uint32_t quad_of(int slot) const { return quad[slot]; }
};
template <int kW>
struct Stage<kW, false> : StageCore<kW> {
    __device__ uint32_t quad_of(int slot) const { return __float_as_uint(this->c[slot].w); }
};

// Minimum of q(u, v) = (l00 u + l10 v)^2 + (l11 v)^2 (positive definite)
// over the rectangle [u0, u1] x [v0, v1]: zero if it holds the origin, else
// the least of the four edges' clamped one-dimensional minima.  The clamp
// points use the expanded coefficients qa = l00^2, qb = l00 l10,
// qc = l10^2 + l11^2 (ra = 1/qa, rc = 1/qc); q itself is evaluated as two
// squares, which stays accurate when the expanded terms would cancel.
__device__ inline float rect_min_quadratic(float l00, float l10, float l11, float qb, float ra, float rc, float u0,
                                           float u1, float v0, float v1) {
    if (u0 <= 0.0f && u1 >= 0.0f && v0 <= 0.0f && v1 >= 0.0f) return 0.0f;
    auto q = [&](float u, float v) {
        const float s = __builtin_fmaf(l10, v, l00 * u), t = l11 * v;
        return __builtin_fmaf(s, s, t * t);
    };
    float best = __builtin_huge_valf();
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float u = e ? u1 : u0;
        best = fminf(best, q(u, fminf(fmaxf(-qb * u * rc, v0), v1)));
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float v = e ? v1 : v0;
        best = fminf(best, q(fminf(fmaxf(-qb * v * ra, u0), u1), v));
    }
    return best;
}

// Stage the record of Gaussian gid in slot `slot` (rdepth: per-record depth
// values, read when kAux).
// qin >= 0: the quadrant mask as an earlier staging of the same instance
// found it (the tests are skipped).  Returns the mask.
template <bool kAux, int kW>
__device__ inline uint32_t stage(const BlendRecord *rec, const float *rdepth, uint32_t gid, float X0, float Y0,
                                 float W, Stage<kW, kAux> &S, int slot, int qin = -1) {
    const float4 *p = reinterpret_cast<const float4 *>(rec + gid);
    const float4 ra4 = p[0], rb4 = p[1], rc4 = p[2];
    float x = (ra4.x - X0) + ra4.y;  // px_hi - X0 is exact near the tile
    const float y = (ra4.z - Y0) + ra4.w;
    // the same centre in double precision: exactly hi - X0 + lo
    double xd = ((double)ra4.x - (double)X0) + (double)ra4.y;
    const double yd = ((double)ra4.z - (double)Y0) + (double)ra4.w;
    // bring the centre within half a turn of the tile's middle column
    const float half = 0.5f * W;
    if (x - 8.0f >= half) {
        x -= W;
        xd -= (double)W;
    }
    if (x - 8.0f < -half) {
        x += W;
        xd += (double)W;
    }
    const float l00 = rb4.x, l10 = rb4.y, l11 = rb4.z;
    // quadrants the alpha >= alpha_min region can reach:
    // |L^T (u, v)|^2 <= log2(o / alpha_min), with a margin; the clamped edge
    // minima only need to be near-exact: a slightly wrong clamp point still
    // bounds the minimum over an edge from above, and the margin absorbs the
    // rounding
    uint32_t quad = (uint32_t)qin;
    if (qin < 0) {
    const float reach = rc4.w + 1e-3f * (1.0f + fabsf(rc4.w));
    const float qa = l00 * l00, qb = l00 * l10, qc = __builtin_fmaf(l10, l10, l11 * l11);
    const float ra = __builtin_amdgcn_rcpf(qa), rc = __builtin_amdgcn_rcpf(qc);
    quad = 0;
#pragma unroll
    for (int k = 0; k < kQuads; ++k) {
        const float qx = (float)((k & 1) * 8), qy = (float)((k >> 1) * 8);
        const float u0 = qx + 0.5f - x, u1 = qx + 7.5f - x;
        const float v0 = qy + 0.5f - y, v1 = qy + 7.5f - y;
        // offsets that the seam wrap may shift: keep the quadrant
        const bool wraps = u0 < -half || u1 >= half;
        if (wraps || rect_min_quadratic(l00, l10, l11, qb, ra, rc, u0, u1, v0, v1) <= reach) quad |= 1u << k;
    }
    }
    // columns whose offset i + 1/2 - x leaves [-W/2, W/2) take the centre a
    // turn away: the right ones (offset >= W/2) or the left ones (< -W/2)
    float thr = 1e30f;
    double xad = xd, xbd = xd;
    if (15.5f - x >= half) {
        xbd = xd + (double)W;
        thr = x + half - 0.5f;
    } else if (0.5f - x < -half) {
        xad = xd - (double)W;
        thr = x - half - 0.5f;
    }
    const double dy0 = 0.5 - yd;
    const float u0a = (float)((double)l00 * (0.5 - xad) + (double)l10 * dy0);
    const float u0b = (float)((double)l00 * (0.5 - xbd) + (double)l10 * dy0);
    const float v0 = (float)((double)l11 * dy0);
    S.a[slot] = make_float4(u0a, v0, l00, l10);
    S.b[slot] = make_float4(l11, rb4.w, rc4.x, rc4.y);
    // bit kSplitBit: the tile's columns take two centres (thr inside the tile)
    const uint32_t qm = quad | (thr < 1e29f ? kSplitBit : 0u);
    S.c[slot] = make_float4(rc4.z, u0b, thr, kAux ? rdepth[gid] : __uint_as_float(qm));
    if constexpr (kAux) S.quad[slot] = qm;
    return quad;
}

// Wave w lists, in order, the staged slots in [lo, nb) that reach one of its
// quadrants; returns the count (uniform) and sets `split` (uniform) when one
// of them has its seam split inside the tile.
template <int kW, bool kAux>
__device__ inline int compact(Stage<kW, kAux> &S, int w, int lo, int nb, bool &split, const int *qlo = nullptr) {
    constexpr int kPPL = kQuads / kW;
    const int lane = __lane_id();
    int n = 0;
    bool sp = false;
    for (int c = 0; c < Stage<kW, kAux>::kBatch; c += kWave) {
        const int slot = c + lane;
        const uint32_t q = (slot >= lo && slot < nb) ? S.quad_of(slot) : 0u;
        uint32_t m = (q >> (w * kPPL)) & ((1u << kPPL) - 1u);
        if (qlo) {
            // per-quadrant lower bounds: quadrant k of this wave drops slots below qlo[k]
#pragma unroll
            for (int k = 0; k < kPPL; ++k)
                if (slot < qlo[k]) m &= ~(1u << k);
        }
        const uint64_t hits = __ballot(m != 0u);
        if (m) S.list[w][n + __popcll(hits & ((1ull << lane) - 1ull))] = (uint16_t)(slot | (m << 8));
        sp |= m != 0u && (q & kSplitBit);
        n += __popcll(hits);
    }
    split = __ballot(sp) != 0ull;
    return n;
}

// alpha at the pixel (i, j) of the tile (integer coordinates as floats):
// returns the unclamped alpha o exp(-1/2 d^T Q d) = 2^(log2 o - |w|^2),
// writes the clamped one and w = (u, v) = L^T d (L scaled as staged).
template <bool kSplit>
__device__ __forceinline__ float pixel_alpha(float i, float j, float4 a, float4 c, float l11, float log2o,
                                             float alpha_max, float &alpha, float &u, float &v) {
    // without a split every column takes u0a (thr lies past the tile)
    const float u0 = (kSplit && i >= c.z) ? c.y : a.x;
    u = __builtin_fmaf(a.z, i, __builtin_fmaf(a.w, j, u0));
    v = __builtin_fmaf(l11, j, a.y);
    const float araw = __builtin_amdgcn_exp2f(__builtin_fmaf(-u, u, __builtin_fmaf(-v, v, log2o)));
    // araw >= 0: non-negative floats order as their bit patterns, so the
    // clamp is an integer min (no canonicalisation of alpha_max per pixel);
    // a NaN araw gives alpha_max or a NaN alpha, which no pixel blends
    alpha = __int_as_float(min(__float_as_int(araw), __float_as_int(alpha_max)));
    return araw;
}

// Pixel (inside the tile) of slot s of wave w, lane (lx, ly) of an 8x8 block.
template <int kW>
__device__ __forceinline__ int slot_px(int w, int s, int lx) { return (((w * (kQuads / kW)) + s) & 1) * 8 + lx; }
template <int kW>
__device__ __forceinline__ int slot_py(int w, int s, int ly) { return (((w * (kQuads / kW)) + s) >> 1) * 8 + ly; }

// kDepth: also the depth image sum_i d_i alpha_i T_i.  kCount: also the
// number of instances blended per pixel (only when a frame asks for it).
template <int kN>
__device__ __forceinline__ bool all_stopped(const float (&T)[kN]) {
    bool a = true;
#pragma unroll
    for (int k = 0; k < kN; ++k) a = a && !(T[k] > 0.0f);
    return a;
}

// Eight waves per SIMD (at most 64 VGPRs) for the four-wave colour-only
// forward: it then fits without spills and hides more of its LDS latency;
// the other instantiations need more registers.
template <int kW, bool kDepth, bool kCount>
constexpr int forward_min_waves() { return (kW == 4 && !kDepth && !kCount) ? 8 : 1; }

template <int kW, bool kBatched, bool kDepth, bool kCount>
__global__ __launch_bounds__(kWave * kW, (forward_min_waves<kW, kDepth, kCount>())) void k_blend_forward(FrameTable FT, const BlendRecord *rec,
                                                               const float *rdepth, const uint32_t *inst_gauss,
                                                               const uint2 *ranges, BlendSettings s,
                                                               const uint32_t *order, uint32_t *tile_work) {
    constexpr int kNT = kWave * kW, kPPL = kQuads / kW, kBatch = Stage<kW, kDepth>::kBatch;
    __shared__ Stage<kW, kDepth> S;
    __shared__ int s_wmax[kW];
    const uint32_t tile = order ? order[blockIdx.x] : blockIdx.x;
    const int fi = kBatched ? find_frame(FT, tile) : 0;
    const BlendFrame &F = FT.f[fi];
    const uint32_t lt = tile - F.tile_base;
    const int tx = lt % F.tiles_x, ty = lt / F.tiles_x;
    const int w = threadIdx.x / kWave, lane = __lane_id();
    const int lx = lane & 7, ly = lane >> 3;
    const float W = F.period;
    const float X0 = (float)(tx * kTile), Y0 = (float)(ty * kTile);
    const uint2 range = ranges[tile];
    const int count = (int)(range.y - range.x);
    float T[kPPL], C0[kPPL], C1[kPPL], C2[kPPL], Dp[kPPL];
    int last[kPPL], blended[kPPL];
    // a pixel that has stopped (or lies outside the image) holds -T: with
    // T <= 0, T (1 - alpha) never passes T_min > 0, so the test that stops a
    // pixel also keeps it stopped, and |T| is its transmittance
#pragma unroll
    for (int k = 0; k < kPPL; ++k) {
        T[k] = 1.0f;
        C0[k] = C1[k] = C2[k] = Dp[k] = 0.0f;
        last[k] = blended[k] = 0;
        if (ty * kTile + slot_py<kW>(w, k, ly) >= F.height || tx * kTile + slot_px<kW>(w, k, lx) >= F.width)
            T[k] = -1.0f;
    }
    for (int base = 0; base < count; base += kBatch) {
        if (__syncthreads_count(all_stopped(T)) == kNT) break;
        const int nb = min(kBatch, count - base);
        if ((int)threadIdx.x < nb) {
            const uint32_t at = range.x + base + threadIdx.x;
            const uint32_t q = stage<kDepth>(rec, rdepth, inst_gauss[at], X0, Y0, W, S, threadIdx.x);
            if (F.quad) F.quad[at] = (uint8_t)q;
        }
        __syncthreads();
        if (__ballot(!all_stopped(T)) == 0ull) continue;  // this wave is finished: keep staging with the others
        bool split;
        const int n = compact(S, w, 0, nb, split);
        // the walk, with the seam split of a centre handled only in batches
        // that hold such an instance (uniform branch)
        auto walk = [&](auto split_tag) {
            constexpr bool kSplit = decltype(split_tag)::value;
            // blend instance t with its record in (a, b, c) (uniform entry e)
            auto blend_one = [&](uint32_t e, const float4 &a, const float4 &b, const float4 &c) {
                const int j = e & 0xff;
                const uint32_t m = e >> 8;
                const float cb = c.x;
                const float dj = c.w;
#pragma unroll
                for (int k = 0; k < kPPL; ++k) {
                    if (!(m & (1u << k))) continue;  // uniform
                    float alpha, u, v;
                    pixel_alpha<kSplit>((float)slot_px<kW>(w, k, lx), (float)slot_py<kW>(w, k, ly), a, c, b.x, b.y,
                                        s.alpha_max, alpha, u, v);
                    const float aT = alpha * T[k];
                    const float Tn = T[k] - aT;  // T (1 - alpha)
                    const bool live = alpha >= s.alpha_min;
                    const bool keep = Tn >= s.T_min;  // false for a stopped pixel (T <= 0)
                    const bool take = live && keep;
                    const float wgt = take ? aT : 0.0f;
                    C0[k] = __builtin_fmaf(b.z, wgt, C0[k]);
                    C1[k] = __builtin_fmaf(b.w, wgt, C1[k]);
                    C2[k] = __builtin_fmaf(cb, wgt, C2[k]);
                    if (kDepth) Dp[k] = __builtin_fmaf(dj, wgt, Dp[k]);
                    // stopping: T keeps its magnitude with the sign flipped
                    T[k] = live ? (keep ? Tn : -fabsf(T[k])) : T[k];
                    last[k] = take ? base + j + 1 : last[k];
                    if (kCount) blended[k] += take ? 1 : 0;
                }
            };
            if constexpr (kW != 4) {
                // two pixels per lane: the registers a second record set
                // would take cost more waves than the latency it hides
                for (int t = 0; t < n; ++t) {
                    const uint32_t e = __builtin_amdgcn_readfirstlane(S.list[w][t]);
                    // the record into registers once (a reference into LDS
                    // would be read again by each quadrant)
                    const float4 a = S.a[e & 0xff], b = S.b[e & 0xff], c = S.c[e & 0xff];
                    blend_one(e, a, b, c);
                    if ((t & 15) == 15 && __ballot(!all_stopped(T)) == 0ull) break;
                }
                return;
            }
            if (n == 0) return;
            // two register sets in turn: the record of the next instance is
            // read from LDS while this one blends
            uint32_t e0 = __builtin_amdgcn_readfirstlane(S.list[w][0]), e1 = 0;
            float4 a0 = S.a[e0 & 0xff], b0 = S.b[e0 & 0xff], c0 = S.c[e0 & 0xff], a1, b1, c1;
            for (int t = 0; t < n; t += 2) {
                if (t + 1 < n) {
                    e1 = __builtin_amdgcn_readfirstlane(S.list[w][t + 1]);
                    a1 = S.a[e1 & 0xff];
                    b1 = S.b[e1 & 0xff];
                    c1 = S.c[e1 & 0xff];
                }
                blend_one(e0, a0, b0, c0);
                if (t + 1 >= n) break;
                if (t + 2 < n) {
                    e0 = __builtin_amdgcn_readfirstlane(S.list[w][t + 2]);
                    a0 = S.a[e0 & 0xff];
                    b0 = S.b[e0 & 0xff];
                    c0 = S.c[e0 & 0xff];
                }
                blend_one(e1, a1, b1, c1);
                if ((t & 15) == 14 && __ballot(!all_stopped(T)) == 0ull) break;
            }
        };
        if (split)
            walk(std::true_type{});
        else
            walk(std::false_type{});
    }
    // the tile's backward walk length: its largest contributor count
    int wmax = 0;
#pragma unroll
    for (int k = 0; k < kPPL; ++k) wmax = max(wmax, last[k]);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) wmax = max(wmax, __shfl_xor(wmax, off, kWave));
    if (lane == 0) s_wmax[w] = wmax;
    __syncthreads();
    if (threadIdx.x == 0 && tile_work) {
        int m = 0;
#pragma unroll
        for (int k = 0; k < kW; ++k) m = max(m, s_wmax[k]);
        tile_work[tile] = (uint32_t)m;
    }
    const int64_t HW = (int64_t)F.width * F.height;
#pragma unroll
    for (int k = 0; k < kPPL; ++k) {
        const int y = ty * kTile + slot_py<kW>(w, k, ly), x = tx * kTile + slot_px<kW>(w, k, lx);
        if (y >= F.height || x >= F.width) continue;
        const int64_t p = (int64_t)y * F.width + x;
        T[k] = fabsf(T[k]);  // a stopped pixel holds -T
        F.image[p] = __builtin_fmaf(T[k], s.bg[0], C0[k]);
        F.image[HW + p] = __builtin_fmaf(T[k], s.bg[1], C1[k]);
        F.image[2 * HW + p] = __builtin_fmaf(T[k], s.bg[2], C2[k]);
        F.final_T[p] = T[k];
        F.n_contrib[p] = last[k];
        if (kCount && F.n_blended) F.n_blended[p] = blended[k];
        if (kDepth) F.depth[p] = Dp[k];
    }
}

template <int kCtrl, int kRowMask>
__device__ __forceinline__ float dpp_add(float v) {
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, kRowMask, 0xF, false));
}

// Reduce-scatter of kNF <= 10 per-lane values over the wave, each exchange
// carrying two fields: permlane32_swap pairs the wave halves (register p:
// field 2p in lanes 0-31, 2p+1 in lanes 32-63), permlane16_swap pairs the
// rows (register q, row r: field 4q + 2(r & 1) + (r >> 1)), then inside each
// 16-lane row two pairing steps (row mirror, half-row mirror: a lane keeps
// one field and sends the other to its partner) and two quad steps.  Lane l
// ends with the wave-wide sum of field rs_field(l) (each field in the four
// lanes l ^ {0, 1, 2, 3}).  Every lane must be active (DPP reads its
// partner).
__device__ __forceinline__ void swap_add(float &x, float &y, bool half32) {
    const auto r = half32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false)
                          : __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    x = __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
template <int kCtrl>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xF, 0xF, false));
}
template <int kCtrl>
__device__ __forceinline__ float pair_step(float a, float b, bool hi) {
    const float keep = hi ? b : a, send = hi ? a : b;
    return keep + dpp_mov<kCtrl>(send);
}
__device__ __forceinline__ int rs_field(int lane) {
    return 8 * ((lane >> 2) & 1) + 4 * ((lane >> 3) & 1) + 2 * ((lane >> 4) & 1) + (lane >> 5);
}
template <int kNF>
__device__ __forceinline__ float wave_reduce_scatter(const float (&v)[kAccAux], int lane) {
    float y[5];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
        float a = 2 * p < kNF ? v[2 * p] : 0.0f, b = 2 * p + 1 < kNF ? v[2 * p + 1] : 0.0f;
        if (2 * p < kNF) swap_add(a, b, true);
        y[p] = a;
    }
    float z0 = y[0], z1 = y[2], z2 = y[4], t1 = y[1], t3 = y[3], zero = 0.0f;
    swap_add(z0, t1, false);
    swap_add(z1, t3, false);
    swap_add(z2, zero, false);
    const bool h8 = lane & 8, h4 = lane & 4;
    const float w0 = pair_step<0x140>(z0, z1, h8);  // row_mirror
    // z2 pairs with an all-zero register: lanes 0-7 of a row sum its fields
    // (8-11); lanes 8-15 would hold fields 12-15, which do not exist, so they
    // take the same sums (no select: every lane takes part in each exchange)
    const float w1 = z2 + dpp_mov<0x140>(z2);
    float u = pair_step<0x141>(w0, w1, h4);  // row_half_mirror
    u = dpp_add<0x4E, 0xF>(u);               // quad_perm [2,3,0,1]
    u = dpp_add<0xB1, 0xF>(u);               // quad_perm [1,0,3,2]
    return u;
}

// kAux: the depth and alpha cotangents too (colour channels with colour
// d_i and 1 over a black background), and a tenth accumulator dL/dd.
template <int kW, bool kBatched, bool kAux>
__global__ __launch_bounds__(kWave * kW) void k_blend_backward(FrameTable FT, const BlendRecord *rec,
                                                                const float *rdepth, const uint32_t *inst_gauss,
                                                                const uint2 *ranges, BlendSettings s, float *acc,
                                                                const uint32_t *order) {
    constexpr int kPPL = kQuads / kW, kBatch = Stage<kW, kAux>::kBatch;
    constexpr int kNF = kAux ? kAccAux : kAcc;  // accumulator fields per Gaussian
    __shared__ Stage<kW, kAux> S;
    __shared__ float part[kBatch][kNF];
    // per-wave contributor maxima, read before the first batch clears part
    int *s_max = reinterpret_cast<int *>(&part[0][0]);
    const uint32_t tile = order ? order[blockIdx.x] : blockIdx.x;
    const int fi = kBatched ? find_frame(FT, tile) : 0;
    const BlendFrame &F = FT.f[fi];
    const uint32_t lt = tile - F.tile_base;
    const int tx = lt % F.tiles_x, ty = lt / F.tiles_x;
    const int w = threadIdx.x / kWave, lane = __lane_id();
    const int lx = lane & 7, ly = lane >> 3;
    const float W = F.period;
    const float X0 = (float)(tx * kTile), Y0 = (float)(ty * kTile);
    const uint2 range = ranges[tile];
    const int64_t HW = (int64_t)F.width * F.height;
    float T[kPPL], dLS[kPPL], dL0[kPPL], dL1[kPPL], dL2[kPPL], dLD[kPPL], dLA[kPPL];
    int last[kPPL];
    int wmax = 0;
#pragma unroll
    for (int k = 0; k < kPPL; ++k) {
        const int y = ty * kTile + slot_py<kW>(w, k, ly), x = tx * kTile + slot_px<kW>(w, k, lx);
        T[k] = 1.0f;
        dL0[k] = dL1[k] = dL2[k] = dLD[k] = dLA[k] = 0.0f;
        last[k] = 0;
        if (y < F.height && x < F.width) {
            const int64_t p = (int64_t)y * F.width + x;
            T[k] = F.final_T[p];
            last[k] = F.n_contrib[p];
            dL0[k] = F.dL[p];
            dL1[k] = F.dL[HW + p];
            dL2[k] = F.dL[2 * HW + p];
            if (kAux) {
                dLD[k] = F.dLD ? F.dLD[p] : 0.0f;
                dLA[k] = F.dLA ? F.dLA[p] : 0.0f;
            }
        }
        // dL . (colour blended behind the current instance + T_final bg)
        dLS[k] = T[k] * (dL0[k] * s.bg[0] + dL1[k] * s.bg[1] + dL2[k] * s.bg[2]);
        wmax = max(wmax, last[k]);
    }
    // per-wave and per-tile maxima of the contributor counts
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) wmax = max(wmax, __shfl_xor(wmax, off, kWave));
    if (lane == 0) s_max[w] = wmax;
    // per-quadrant largest contributor counts of this wave: a quadrant skips
    // the positions past its own pixels' last contributors
    int qmax[kPPL];
#pragma unroll
    for (int k = 0; k < kPPL; ++k) {
        int m = last[k];
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) m = max(m, __shfl_xor(m, off, kWave));
        qmax[k] = __builtin_amdgcn_readfirstlane(m);
    }
    __syncthreads();
    int max_last = 0;
#pragma unroll
    for (int k = 0; k < kW; ++k) max_last = max(max_last, s_max[k]);
    for (int hi = max_last; hi > 0; hi -= kBatch) {
        const int nb = min(kBatch, hi);
        __syncthreads();
        uint32_t my_gid = 0;  // the Gaussian this thread stages (slot threadIdx.x)
        if ((int)threadIdx.x < nb) {
            // slot i holds list position hi-1-i (staged by the forward, which
            // left the quadrant mask of every position it staged)
            const uint32_t at = range.x + hi - 1 - threadIdx.x;
            my_gid = inst_gauss[at];
            stage<kAux>(rec, rdepth, my_gid, X0, Y0, W, S, threadIdx.x, F.quad ? (int)F.quad[at] : -1);
#pragma unroll
            for (int f = 0; f < kNF; ++f) part[threadIdx.x][f] = 0.0f;
        }
        __syncthreads();
        // positions at or past this wave's largest contributor count (slots
        // below hi - wmax) are never blended by its pixels, and positions past
        // quadrant k's largest count (slots below hi - qmax[k]) by that
        // quadrant's
        bool split;
        int qlo[kPPL];
#pragma unroll
        for (int k = 0; k < kPPL; ++k) qlo[k] = hi - qmax[k];
        const int n = compact(S, w, hi - wmax, nb, split, qlo);
        auto walk = [&](auto split_tag) {
            constexpr bool kSplit = decltype(split_tag)::value;
            for (int t = 0; t < n; ++t) {
                const uint32_t e = __builtin_amdgcn_readfirstlane(S.list[w][t]);
                const int j = e & 0xff;
                const uint32_t m = e >> 8;
                const int pos = hi - 1 - j;
                const float4 a = S.a[j], b = S.b[j], c = S.c[j];
                const float cb = c.x;
                const float dj = c.w;
                float v[kAccAux];
#pragma unroll
                for (int f = 0; f < kAccAux; ++f) v[f] = 0.0f;
                bool any = false;  // uniform: some lane blends this instance
#pragma unroll
                for (int k = 0; k < kPPL; ++k) {
                    if (!(m & (1u << k))) continue;  // uniform
                    const float fi = (float)slot_px<kW>(w, k, lx), fj = (float)slot_py<kW>(w, k, ly);
                    float alpha, wu, wv;
                    const float araw = pixel_alpha<kSplit>(fi, fj, a, c, b.x, b.y, s.alpha_max, alpha, wu, wv);
                    const bool valid = pos < last[k] && alpha >= s.alpha_min;
                    if (__ballot(valid) == 0ull) continue;  // uniform: nothing blended in this quadrant
                    any = true;
                    // a lane that does not blend this instance takes alpha = 0:
                    // 1 / (1 - 0) = 1 exactly, so its T stays as it is and its
                    // weight and colour terms are zero
                    const float ae = valid ? alpha : 0.0f;
                    const float inv = __builtin_amdgcn_rcpf(1.0f - ae);
                    const float Tf = T[k] * inv;  // transmittance in front of this instance
                    T[k] = Tf;
                    const float wgt = ae * Tf;
                    float dLc = __builtin_fmaf(dL0[k], b.z, __builtin_fmaf(dL1[k], b.w, dL2[k] * cb));
                    if (kAux) dLc += __builtin_fmaf(dLD[k], dj, dLA[k]);  // depth and alpha channels
                    const float dalpha = __builtin_fmaf(dLc, Tf, -(dLS[k] * inv));
                    dLS[k] = __builtin_fmaf(dLc, wgt, dLS[k]);
                    v[6] = __builtin_fmaf(dL0[k], wgt, v[6]);
                    v[7] = __builtin_fmaf(dL1[k], wgt, v[7]);
                    v[8] = __builtin_fmaf(dL2[k], wgt, v[8]);
                    if (kAux) v[9] = __builtin_fmaf(dLD[k], wgt, v[9]);
                    // dL/dalpha through an unclamped alpha only
                    const float da = (valid && araw < s.alpha_max) ? dalpha : 0.0f;
                    // moments of gp = dL/d(-1/2 d^T Q d) = alpha * dL/dalpha over
                    // w = (wu, wv) = L^T d, which the exponent has formed already
                    const float gp = araw * da;
                    const float gu = wu * gp, gv = wv * gp;
                    v[0] += gu;
                    v[1] += gv;
                    v[2] = __builtin_fmaf(wu, gu, v[2]);
                    v[3] = __builtin_fmaf(wu, gv, v[3]);
                    v[4] = __builtin_fmaf(wv, gv, v[4]);
                    v[5] += gp;  // o dL/do
                }
                if (any) {
                    const float u = wave_reduce_scatter<kNF>(v, lane);
                    const int f = rs_field(lane);
                    if ((lane & 3) == 0 && f < kNF) {
                        if (kW == 1) part[j][f] = u;
                        else atomicAdd(&part[j][f], u);  // the waves of this instance meet here
                    }
                }
            }
        };
        if (split)
            walk(std::true_type{});
        else
            walk(std::false_type{});
        __syncthreads();
        // moments -> screen-space gradients: the staging lane of each slot
        if ((int)threadIdx.x < nb && (S.quad_of(threadIdx.x) & ~kSplitBit)) {
            const int j = threadIdx.x;
            float mo[kNF];
#pragma unroll
            for (int f = 0; f < kNF; ++f) mo[f] = part[j][f];
            // Q = 2 ln2 L L^T (L scaled by sqrt(log2(e) / 2)), so
            // dL/dp = Q sum(d gp) = 2 ln2 L sum(w gp) with w = L^T d; the
            // second moments sum(w w^T gp) go out as they are
            const float4 a = S.a[j], b = S.b[j];
            const float l00 = a.z, l10 = a.w, l11 = b.x;
            float out[kNF];
            out[0] = 2.0f * kLn2 * (l00 * mo[0]);                          // dL/dp_x
            out[1] = 2.0f * kLn2 * __builtin_fmaf(l10, mo[0], l11 * mo[1]);  // dL/dp_y
            out[2] = mo[2];  // sum(wu wu gp)
            out[3] = mo[3];  // sum(wu wv gp)
            out[4] = mo[4];  // sum(wv wv gp)
            out[5] = mo[5] * __builtin_amdgcn_exp2f(-b.y);  // dL/do: sum(gp) / o
            out[6] = mo[6];
            out[7] = mo[7];
            out[8] = mo[8];
            if (kAux) out[kNF - 1] = mo[kNF - 1];  // dL/dd
#pragma unroll
            for (int f = 0; f < kNF; ++f) part[j][f] = out[f];
        }
        __syncthreads();
        // each wave walks the fields of the slots it staged in order, so the
        // lanes of one atomic instruction cover whole records of a few
        // Gaussians (a handful of cache lines) rather than one field of 64
        // scattered Gaussians (64 lines): L2 takes far fewer atomic requests;
        // a slot's Gaussian id comes from the lane that staged it
        const int j0 = w * kWave;
        const int nq = max(0, min(kWave, nb - j0)) * kNF;
        const float *flat = &part[j0][0];
#pragma unroll 1
        for (int i = 0; i < kNF; ++i) {
            const int q = lane + i * kWave, jl = q / kNF, f = q - jl * kNF;
            const uint32_t g = (uint32_t)__shfl((int)my_gid, jl, kWave);
            const float val = q < nq ? flat[q] : 0.0f;
            if (val != 0.0f) atomicAdd(acc + (int64_t)g * kNF + f, val);
        }
    }
}

constexpr int kOrderThreads = 1024;

__global__ __launch_bounds__(kOrderThreads) void k_tile_order(const uint2 *ranges, const uint32_t *work,
                                                              uint32_t ntiles, uint32_t *order) {
    __shared__ TileOrderShared sh;
    tile_order_block<kOrderThreads>(ranges, work, ntiles, order, sh);
}

// Workgroup 0 writes the tile order (it starts first, and its loads and LDS
// passes run beside the clearing); the others clear four words per thread.
__global__ __launch_bounds__(kOrderThreads) void k_clear_and_order(uint32_t *acc, int64_t n, const uint32_t *work,
                                                                   uint32_t ntiles, uint32_t *order) {
    __shared__ TileOrderShared sh;
    if (blockIdx.x == 0) {
        if (ntiles > 0) tile_order_block<kOrderThreads>(nullptr, work, ntiles, order, sh);
        return;
    }
    const int64_t i = ((int64_t)(blockIdx.x - 1) * kOrderThreads + threadIdx.x) * 4;
    if (i + 4 <= n && (reinterpret_cast<uintptr_t>(acc + i) & 15u) == 0) {
        *reinterpret_cast<uint4 *>(acc + i) = make_uint4(0u, 0u, 0u, 0u);
    } else {
        for (int64_t k = i; k < i + 4 && k < n; ++k) acc[k] = 0u;
    }
}

float period_of(const FrameGeom &f) { return f.wrap ? (float)f.width : __builtin_huge_valf(); }

}  // namespace

hipError_t launch_tile_order(const uint2 *ranges, const uint32_t *work, uint32_t ntiles, uint32_t *order,
                             hipStream_t st) {
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, st, ranges, work, ntiles, order);
    return hipGetLastError();
}

hipError_t launch_clear_and_order(uint32_t *acc, int64_t n, const uint32_t *work, uint32_t ntiles, uint32_t *order,
                                  hipStream_t st) {
    if (n < 0 || (ntiles > 0 && !work)) return hipErrorInvalidValue;
    const int64_t fill_blocks = (n + 4 * kOrderThreads - 1) / (4 * kOrderThreads);
    hipLaunchKernelGGL(k_clear_and_order, dim3((unsigned)(1 + fill_blocks)), dim3(kOrderThreads), 0, st, acc, n, work,
                       ntiles, order);
    return hipGetLastError();
}

template <int kW>
void launch_forward_waves(const FrameTable &T, unsigned tiles, const BlendRecord *rec, const float *rdepth,
                          const uint32_t *inst_gauss, const uint2 *ranges, const BlendSettings &s, bool depth,
                          const uint32_t *order, uint32_t *tile_work, hipStream_t st) {
    const float *rd = depth ? rdepth : nullptr;
    const bool count = T.f[0].n_blended != nullptr;
    if (depth && count)
        hipLaunchKernelGGL((k_blend_forward<kW, false, true, true>), dim3(tiles), dim3(kWave * kW), 0, st, T, rec, rd,
                           inst_gauss, ranges, s, order, tile_work);
    else if (depth)
        hipLaunchKernelGGL((k_blend_forward<kW, false, true, false>), dim3(tiles), dim3(kWave * kW), 0, st, T, rec,
                           rd, inst_gauss, ranges, s, order, tile_work);
    else if (count)
        hipLaunchKernelGGL((k_blend_forward<kW, false, false, true>), dim3(tiles), dim3(kWave * kW), 0, st, T, rec,
                           rd, inst_gauss, ranges, s, order, tile_work);
    else
        hipLaunchKernelGGL((k_blend_forward<kW, false, false, false>), dim3(tiles), dim3(kWave * kW), 0, st, T, rec,
                           rd, inst_gauss, ranges, s, order, tile_work);
}

// Mean instances per tile above which two waves per tile (two pixels per
// lane: each staged instance's LDS reads and scalar work shared by two
// pixels) beat four (shorter walks per wave); measured 0.51 -> 0.46 ms at
// 5.8k per tile, 0.27 -> 0.31 ms the other way at 1.4k.  Every pixel's
// arithmetic is the same either way.  With such lists the longest-first
// launch order no longer shortens the forward (0.453 vs 0.448 ms at 5.8k;
// 0.26 vs 0.31 ms at 1.4k), so the forward then runs in tile order.
constexpr uint64_t kLongLists = 3000;

bool forward_uses_order(uint64_t instances, uint32_t tiles) { return instances <= kLongLists * (uint64_t)tiles; }

hipError_t launch_blend_forward(const FrameGeom &f, const BlendRecord *rec, const float *rdepth,
                                const uint32_t *inst_gauss, const uint2 *ranges, const BlendSettings &s, float *image,
                                float *final_T, int32_t *n_contrib, int32_t *n_blended, float *depth_out,
                                const uint32_t *order, uint32_t *tile_work, uint64_t instances, hipStream_t st,
                                uint8_t *inst_quad) {
    FrameTable T{};
    T.n = 1;
    T.f[0] = BlendFrame{f.width, f.height, f.tiles_x, f.tiles_y, 0u, period_of(f), image, final_T, n_contrib,
                        n_blended, nullptr, depth_out, nullptr, nullptr, inst_quad};
    const unsigned tiles = (unsigned)(f.tiles_x * f.tiles_y);
    if (tiles == 0) return hipSuccess;
    if (instances > kLongLists * tiles)
        launch_forward_waves<2>(T, tiles, rec, rdepth, inst_gauss, ranges + f.tile_base, s, depth_out != nullptr,
                                order, tile_work, st);
    else
        launch_forward_waves<OMNIGS_FWD_WAVES>(T, tiles, rec, rdepth, inst_gauss, ranges + f.tile_base, s,
                                               depth_out != nullptr, order, tile_work, st);
    return hipGetLastError();
}

hipError_t launch_blend_forward_frames(const FrameGeom *frames, const omnigs_image_out *outs, int count,
                                       const BlendRecord *rec, const float *rdepth, const uint32_t *inst_gauss,
                                       const uint2 *ranges, const BlendSettings &s, const uint32_t *order,
                                       uint32_t total_tiles, hipStream_t st) {
    if (count < 1 || count > kMaxBatch) return hipErrorInvalidValue;
    if (total_tiles == 0) return hipSuccess;
    FrameTable T{};
    T.n = count;
    bool any_depth = false, any_count = false;
    for (int k = 0; k < count; ++k) {
        const FrameGeom &f = frames[k];
        T.f[k] = BlendFrame{f.width, f.height, f.tiles_x, f.tiles_y, f.tile_base, period_of(f), outs[k].image,
                            outs[k].final_T, outs[k].n_contrib, outs[k].n_blended, nullptr, outs[k].depth,
                            nullptr, nullptr};
        any_depth |= outs[k].depth != nullptr;
        any_count |= outs[k].n_blended != nullptr;
    }
    constexpr int kW = OMNIGS_FWD_WAVES;
    if (any_depth) {
        // every frame then needs a depth buffer
        for (int k = 0; k < count; ++k)
            if (!T.f[k].depth) return hipErrorInvalidValue;
        if (any_count)
            hipLaunchKernelGGL((k_blend_forward<kW, true, true, true>), dim3(total_tiles), dim3(kWave * kW), 0, st, T,
                               rec, rdepth, inst_gauss, ranges, s, order, (uint32_t *)nullptr);
        else
            hipLaunchKernelGGL((k_blend_forward<kW, true, true, false>), dim3(total_tiles), dim3(kWave * kW), 0, st,
                               T, rec, rdepth, inst_gauss, ranges, s, order, (uint32_t *)nullptr);
    } else if (any_count) {
        hipLaunchKernelGGL((k_blend_forward<kW, true, false, true>), dim3(total_tiles), dim3(kWave * kW), 0, st, T,
                           rec, (const float *)nullptr, inst_gauss, ranges, s, order, (uint32_t *)nullptr);
    } else {
        hipLaunchKernelGGL((k_blend_forward<kW, true, false, false>), dim3(total_tiles), dim3(kWave * kW), 0, st, T,
                           rec, (const float *)nullptr, inst_gauss, ranges, s, order, (uint32_t *)nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_blend_backward(const FrameGeom &f, const BlendRecord *rec, const float *rdepth,
                                 const uint32_t *inst_gauss, const uint2 *ranges, const BlendSettings &s,
                                 const float *final_T, const int32_t *n_contrib, const float *dL_dimage,
                                 const float *dL_ddepth, const float *dL_dalpha, float *acc, const uint32_t *order,
                                 hipStream_t st, const uint8_t *inst_quad) {
    FrameTable T{};
    T.n = 1;
    T.f[0] = BlendFrame{f.width, f.height, f.tiles_x, f.tiles_y, 0u, period_of(f), nullptr,
                        const_cast<float *>(final_T), const_cast<int32_t *>(n_contrib), nullptr, dL_dimage, nullptr,
                        dL_ddepth, dL_dalpha, const_cast<uint8_t *>(inst_quad)};
    const unsigned tiles = (unsigned)(f.tiles_x * f.tiles_y);
    if (tiles == 0) return hipSuccess;
    constexpr int kW = OMNIGS_BWD_WAVES;
    if (dL_ddepth || dL_dalpha)
        hipLaunchKernelGGL((k_blend_backward<kW, false, true>), dim3(tiles), dim3(kWave * kW), 0, st, T, rec, rdepth,
                           inst_gauss, ranges + f.tile_base, s, acc, order);
    else
        hipLaunchKernelGGL((k_blend_backward<kW, false, false>), dim3(tiles), dim3(kWave * kW), 0, st, T, rec,
                           (const float *)nullptr, inst_gauss, ranges + f.tile_base, s, acc, order);
    return hipGetLastError();
}

}  // namespace omnigs
