// internal.h -- definitions shared by the HIP translation units of libomnigs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/omnigs.h"

namespace omnigs {

constexpr int kTile = 16;            // tile edge in pixels
constexpr int kTilePixels = kTile * kTile;
constexpr int kBlendThreads = 256;   // one lane per pixel of a 16x16 tile
constexpr int kWave = 64;            // CDNA wavefront
constexpr int kMaxBatch = OMNIGS_MAX_BATCH;  // cameras per batched launch

// Blend record of one Gaussian, 48 bytes: what the blend kernels gather per
// (tile, instance).  The pixel position is split into a float hi part and a
// float lo remainder (p = hi + lo to ~1e-12 px) so that pixel offsets formed
// next to a tile keep full precision at 4K widths.
struct alignas(16) BlendRecord {
    float px_hi, px_lo, py_hi, py_lo;  // pixel position of the centre (Eq. 5 or Eq. 2)
    float l00, l10, l11, log2o;        // Cholesky factor L of Q = Sigma2D^-1 (Eq. 8), scaled by
                                       // sqrt(log2(e) / 2), and log2 of the opacity: the blends
                                       // take alpha = 2^(log2o - |L^T d|^2)
    float r, g, b;                     // SH colour, clamped at 0
    float reach;                       // log2(opacity / alpha_min): alpha >= alpha_min
                                       // iff |L^T d|^2 <= reach (L scaled as above)
};
static_assert(sizeof(BlendRecord) == 48, "record layout");

// Per-Gaussian screen-space gradient accumulators written by the backward
// blend: dL/dp (2); the second moments sum(w w^T gp) (uu, uv, vv) of the
// exponent's cotangent gp = dL/d(-1/2 d^T Q d) over w = Ls^T d, Ls the
// record's scaled factor of Q = Sigma2D^-1 (the projection backward turns
// them into dL/dSigma2D); dL/do, dL/drgb (3); with the depth / alpha
// cotangents a tenth, dL/dd (the Gaussian's depth value).
constexpr int kAcc = 9;
constexpr int kAccAux = 10;

// Depth-sort key of a culled Gaussian: sorts after every finite depth.
constexpr uint32_t kCulledKey = 0xffffffffu;

struct ProjectArgs {
    const float *means, *scales, *quats, *opacities, *sh;
    int64_t n;
    int sh_degree, sh_coeffs;
    double R[9], t[3], campos[3];
    int width, height, tiles_x, tiles_y;
    int rows;                  // rendered rows (<= height; tiles_y covers them)
    int model;                 // OMNIGS_CAMERA_ERP or OMNIGS_CAMERA_PINHOLE
    double fx, fy, cx, cy;     // pinhole intrinsics (Eq. 2)
    double alpha_min, dilation, near_plane;
};

struct FrameGeom {  // one camera's image inside a (possibly batched) launch
    int width, height, tiles_x, tiles_y;
    uint32_t tile_base;  // first global tile id of this image
    int wrap;            // x offsets wrap modulo the width (the ERP seam)
};

// Camera-dependent part of ProjectArgs, one entry per camera of a batch.
struct CamGeom {
    double R[9], t[3], campos[3];
    int width, height, tiles_x, tiles_y, rows;
    int model;
    double fx, fy, cx, cy;
};
struct CamTable {
    int count;
    CamGeom c[kMaxBatch];
};

// Two-level binning: super-tiles of 8x8 tiles.  A record first gets one
// entry per super-tile its tile rectangle touches; each super-tile's list is
// then expanded into the lists of its 64 tiles.
constexpr int kSuper = 8;

// Super-tile rectangle (packed like the tile rectangle: x0 | n_x << 16,
// y0 | n_y << 16; columns wrap modulo ceil(tiles_x / 8)) of the super-tiles
// that the tile rectangle r touches.  When the two pieces of a rectangle
// that wraps across the seam meet in one super-tile column, every column is
// taken; each is still touched (such a rectangle misses fewer than 8 tile
// columns, never the last one), so every super-tile of the rectangle holds
// at least one covered tile.
__host__ __device__ inline uint2 super_rect(uint2 r, int tiles_x) {
    const uint32_t ntx = r.x >> 16, tx0 = r.x & 0xffffu, nty = r.y >> 16, ty0 = r.y & 0xffffu;
    if (ntx == 0 || nty == 0) return make_uint2(0u, 0u);
    const uint32_t tx = (uint32_t)tiles_x, sxn = (tx + kSuper - 1) / kSuper;
    const uint32_t sy0 = ty0 / kSuper, sy1 = (ty0 + nty - 1) / kSuper;
    uint32_t sx0, nsx;
    if (ntx >= tx) {
        sx0 = 0;
        nsx = sxn;
    } else if (tx0 + ntx <= tx) {
        sx0 = tx0 / kSuper;
        nsx = (tx0 + ntx - 1) / kSuper - sx0 + 1;
    } else {
        const uint32_t a0 = tx0 / kSuper, b1 = (tx0 + ntx - 1 - tx) / kSuper;
        if (b1 >= a0) {
            sx0 = 0;
            nsx = sxn;
        } else {
            sx0 = a0;
            nsx = (sxn - a0) + b1 + 1;
        }
    }
    return make_uint2(sx0 | (nsx << 16), sy0 | ((sy1 - sy0 + 1) << 16));
}

// Rows and columns of super-tile (sx, sy) covered by the tile rectangle r
// (columns wrapping across the seam): the covered tiles are their product,
// tile (row k, column c) being tile 8k + c of the super-tile.
struct Cover {
    uint32_t rows, cols;
};
// Bits [lo, hi) of the super-tile starting at column (or row) `base` that
// the tile interval [a, b) covers.
__device__ inline uint32_t cover_span(int a, int b, int base) {
    const int lo = max(a, base) - base, hi = min(b, base + kSuper) - base;
    return hi > lo ? ((1u << hi) - 1u) & ~((1u << lo) - 1u) : 0u;
}
__device__ inline Cover cover_of(uint2 r, int tiles_x, int sx, int sy) {
    const int ntx = (int)(r.x >> 16), tx0 = (int)(r.x & 0xffffu), nty = (int)(r.y >> 16), ty0 = (int)(r.y & 0xffffu);
    const uint32_t rows = cover_span(ty0, ty0 + nty, sy * kSuper);
    if (ntx == 0 || rows == 0u) return Cover{0u, 0u};
    // columns [tx0, tx0 + ntx) modulo tiles_x: the whole row of tiles, one
    // interval, or two when the rectangle wraps across the seam
    const int base = sx * kSuper;
    uint32_t cols;
    if (ntx >= tiles_x)
        cols = cover_span(0, tiles_x, base);
    else if (tx0 + ntx <= tiles_x)
        cols = cover_span(tx0, tx0 + ntx, base);
    else
        cols = cover_span(tx0, tiles_x, base) | cover_span(0, tx0 + ntx - tiles_x, base);
    return Cover{rows, cols};
}

// Block entries' sort keys: the super-tile id, and above it, when every id
// of the launch fits in the 16 bits below (at most kMaxCoverKeyBlocks
// super-tiles), the entry's covered rows | columns << 8, which the radix
// sort (on the id bits only) carries to the binning for free.
constexpr int kCoverShift = 16;
constexpr uint32_t kMaxCoverKeyBlocks = 1u << kCoverShift;
__device__ inline uint32_t cover_bits(Cover c) { return (c.rows | (c.cols << kSuper)) << kCoverShift; }
__device__ inline Cover cover_from_key(uint32_t key) {
    return Cover{(key >> kCoverShift) & ((1u << kSuper) - 1u), key >> (kCoverShift + kSuper)};
}

// Grid geometry of the cameras behind record index g = b * n_per + i, for
// emission into tiles (super == 0: cols = tiles_x, base = first tile id) or
// super-tiles (super == 1: cols = ceil(tiles_x / 8), base = first super id).
struct EmitFrames {
    int64_t n_per;  // records per camera
    int count;
    int super;
    int cover_key;  // super: keys carry the covered rows and columns (kCoverShift)
    int tiles_x[kMaxBatch];
    int cols[kMaxBatch];
    uint32_t base[kMaxBatch];
};

// Tile and super-tile grids of the images of a (possibly batched) launch.
struct SuperFrame {
    uint32_t super_base, tile_base;
    int super_x, super_y, tiles_x, tiles_y;
};
struct SuperTable {
    int count;
    SuperFrame f[kMaxBatch];
};

// Host-side launchers (each .hip file owns its kernels).
// Per record: blend record, depth key, depth value (t_r or t_z; depth may
// be null), tiles covered, tile rectangle, super-tiles touched and screen
// radius (radii may be null); *tiles_total (device) receives the sum of the
// tiles covered (M).
hipError_t launch_project(const ProjectArgs &a, BlendRecord *rec, uint32_t *depth_key, float *depth, uint32_t *n_tiles,
                          uint2 *rect, uint32_t *n_super, float *radii, uint32_t *tiles_total, hipStream_t st,
                          bool cleared = false);
// All cameras of `cams` in one launch: the outputs of camera b for Gaussian i
// land at index b * a.n + i, bit-identical to launch_project of that camera
// (a's camera fields are ignored).
hipError_t launch_project_batch(const ProjectArgs &a, const CamTable &cams, BlendRecord *rec, uint32_t *depth_key,
                                float *depth, uint32_t *n_tiles, uint2 *rect, uint32_t *n_super,
                                uint32_t *tiles_total, hipStream_t st);
// acc: [n][acc_stride] accumulators, acc_stride kAcc or kAccAux.
hipError_t launch_project_backward(const ProjectArgs &a, const uint32_t *n_tiles, const float *acc, int acc_stride,
                                   const omnigs_grads &gr, hipStream_t st);

// radix sort of (u32 key, u32 value) pairs on the low `bits` bits of the key;
// stable.  Result lands in keys_out/vals_out.  vals_in == nullptr sorts the
// input positions 0..n-1 as values.  `scratch` from sort_scratch_bytes.
// n_dev (device, may be null): the element count is min(n, *n_dev), read on
// the device (n then only bounds the buffers and the grid).  n < 2^31 - 1,
// else hipErrorInvalidValue.  key_ranges (device, may be null; only with
// bits <= 8 and n_ranges <= 256): receives [start, end) of each key value
// 0 .. n_ranges-1 in the sorted output.
// cleared: the first sort_clear_words(n, bits) words of `scratch` are
// already zero (the sort then launches no clear of its own).
size_t sort_scratch_bytes(int64_t n);
int64_t sort_clear_words(int64_t n, int bits);
hipError_t radix_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_tmp,
                            uint32_t *vals_tmp, uint32_t *keys_out, uint32_t *vals_out, int64_t n, int bits,
                            void *scratch, hipStream_t st, const uint32_t *n_dev = nullptr,
                            uint2 *key_ranges = nullptr, int n_ranges = 0, bool cleared = false,
                            uint32_t *fault = nullptr);

// Exclusive scan of u32 (optionally of in[gather[i]]); *total (device, may be
// null) receives the sum.  `scratch` from scan_scratch_bytes; cleared: its
// first scan_clear_words(n) words are already zero.
size_t scan_scratch_bytes(int64_t n);
int64_t scan_clear_words(int64_t n);
// The emission's partition, written by the scan of the block-entry counts
// when `part` is given: part[b] = the rank whose output range holds output
// b * (outputs per emit block), for every b < blocks whose output lies below
// the total (as launch_emit's own partition kernel writes it).
struct ScanPartition {
    uint32_t *part = nullptr;
    uint64_t blocks = 0;
};
hipError_t scan_exclusive(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total, void *scratch,
                          hipStream_t st, const uint32_t *gather, bool cleared = false, uint32_t *fault = nullptr,
                          ScanPartition P = {});

// Lookback self-test: the poll bound of every later lookback wait (the
// default is restored by passing 0).  Only the self-test entry point lowers
// it, to make waits give up on purpose.
void set_lookback_poll_limit(uint32_t polls);
// Self-test input: keys[i] = selftest_key(i) & mask.
__host__ __device__ inline uint32_t selftest_key(uint32_t i) {
    uint32_t h = i * 2654435761u + 0x9e3779b9u;
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    return h;
}
hipError_t launch_selftest_keys(uint32_t *keys, int64_t n, uint32_t mask, hipStream_t st);

// Zeroes up to kMaxClear regions of u32 words in one launch (the lookback
// words and counters of the sorts and scans of a call).
constexpr int kMaxClear = 8;
struct ClearList {
    uint32_t *p[kMaxClear];
    int64_t n[kMaxClear];
    int count;
    void add(void *ptr, int64_t words) {
        if (ptr && words > 0 && count < kMaxClear) {
            p[count] = static_cast<uint32_t *>(ptr);
            n[count++] = words;
        }
    }
};
hipError_t launch_clear(const ClearList &L, hipStream_t st);

// Emission in depth order: offs[r] = exclusive scan of the per-record counts
// (tiles or super-tiles, as frames.super says) in depth order, their total M
// at *m_dev (a record's count is the difference of adjacent offsets; a culled
// record's rectangle is empty).  Writes min(M, capacity) (grid id, record) pairs, with global grid
// ids (frames.base of the record's camera plus the id inside its grid); sets
// *overflow when M > capacity.  `part` holds emit_blocks(capacity) entries of
// scratch.
uint64_t emit_blocks(uint64_t capacity);
hipError_t launch_emit(const uint32_t *order, const uint2 *rect, const uint32_t *offs, int64_t n, uint32_t *part,
                       const uint32_t *m_dev, const EmitFrames &frames, uint64_t capacity, uint32_t *inst_tile,
                       uint32_t *inst_gauss, int32_t *overflow, hipStream_t st, bool partitioned = false);
// key_mask: the id bits of the sorted keys.
hipError_t launch_tile_ranges(const uint32_t *inst_tile, const uint32_t *m_dev, uint64_t capacity,
                              uint2 *ranges, uint32_t n_tiles_total, uint32_t key_mask, hipStream_t st);

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);

// Second level of the binning: expands the super-tile lists (sorted by
// super-tile, each in depth order; sranges [start, end) per super-tile)
// into per-tile lists of record ids in depth order, written once each to
// inst_gauss, and fills the [start, end) range of every tile.  Tiles are laid
// out super-tile by super-tile.  super_count (device) is the number of valid
// super entries (at most super_cap).  Instances past inst_cap are dropped and
// set *overflow (may be null); ranges are clamped to inst_cap.  Scratch from
// binning_scratch_bytes.
// binning_clear adds to L the scratch words that a launch with
// cleared == true expects zero.
size_t binning_scratch_bytes(uint64_t super_cap, uint32_t n_super_total);
void binning_clear(void *scratch, uint64_t super_cap, uint32_t n_super_total, ClearList &L);
// skeys: the sorted block-entry keys when they carry the covers (else null:
// the covers come from the Gaussians' rectangles).  fault: the call's
// lookback fault word; with overflow given, a nonzero word sets bit 1 of
// *overflow (bit 0: an instance beyond inst_cap was dropped).  order: when
// given, also the blend's longest-first launch order of the order_tiles
// tiles from the ranges (one workgroup of the expansion).
hipError_t launch_binning(const SuperTable &T, uint32_t n_super_total, const uint2 *rect, const uint32_t *skeys,
                          const uint32_t *sinst_gauss, const uint2 *sranges, uint64_t super_cap, uint64_t inst_cap,
                          void *scratch, uint2 *ranges,
                          uint32_t *inst_gauss, int32_t *overflow, hipStream_t st, bool cleared = false,
                          uint32_t *fault = nullptr, uint32_t *order = nullptr, uint32_t order_tiles = 0);
// *overflow |= 2 when *fault is nonzero (one thread; launch_binning's path
// when there are no blocks).
hipError_t launch_merge_fault(const uint32_t *fault, int32_t *overflow, hipStream_t st);

// Blend kernels.
struct BlendSettings {
    float alpha_min, alpha_max, T_min;
    float bg[3];
};
// `order` (device, may be null): launch order of the tiles (a permutation).
// The forward writes each tile's largest contributor count (the backward's
// walk length) to tile_work (may be null).  With depth_out, the depth image
// from the per-record depth values rdepth.
// Whether launch_blend_forward with `instances` instances over `tiles`
// tiles wants the longest-first launch order (else order may be null).
bool forward_uses_order(uint64_t instances, uint32_t tiles);
hipError_t launch_blend_forward(const FrameGeom &f, const BlendRecord *rec, const float *rdepth,
                                const uint32_t *inst_gauss, const uint2 *ranges, const BlendSettings &s, float *image,
                                float *final_T, int32_t *n_contrib, int32_t *n_blended, float *depth_out,
                                const uint32_t *order, uint32_t *tile_work, uint64_t instances, hipStream_t st,
                                uint8_t *inst_quad = nullptr);
// Forward blend of several images in one launch over their concatenated
// tile space (frames[k].tile_base ascending, total_tiles in all).
hipError_t launch_blend_forward_frames(const FrameGeom *frames, const omnigs_image_out *outs, int count,
                                       const BlendRecord *rec, const float *rdepth, const uint32_t *inst_gauss,
                                       const uint2 *ranges, const BlendSettings &s, const uint32_t *order,
                                       uint32_t total_tiles, hipStream_t st);
// inst_quad (may be null): one byte per tile instance, the reach mask of
// its tile's four 8x8 quadrants, written by the forward for every instance
// it stages and read by the backward (which stages only such instances).
// With dL_ddepth or dL_dalpha (either may be null) the accumulators have
// kAccAux fields per Gaussian, else kAcc; rdepth is read only then.
hipError_t launch_blend_backward(const FrameGeom &f, const BlendRecord *rec, const float *rdepth,
                                 const uint32_t *inst_gauss, const uint2 *ranges, const BlendSettings &s,
                                 const float *final_T, const int32_t *n_contrib, const float *dL_dimage,
                                 const float *dL_ddepth, const float *dL_dalpha, float *acc, const uint32_t *order,
                                 hipStream_t st, const uint8_t *inst_quad = nullptr);
// Longest-first tile order from the list lengths (work == null) or from a
// per-tile work array.  One workgroup; ntiles unbounded.
hipError_t launch_tile_order(const uint2 *ranges, const uint32_t *work, uint32_t ntiles, uint32_t *order,
                             hipStream_t st);
// The backward's set-up in one launch: the gradient accumulators acc[0, n)
// cleared, and the tile order from the recorded walk lengths `work`.
hipError_t launch_clear_and_order(uint32_t *acc, int64_t n, const uint32_t *work, uint32_t ntiles, uint32_t *order,
                                  hipStream_t st);

// Launch order, longest first: tiles bucketed by descending work (work
// clamped to kOrderBuckets - 1) by one workgroup of NT threads (a counting
// sort in LDS), so that the longest walks start first and do not trail the
// blend.  Work is the list length (ranges, work null) or a recorded walk
// length per tile (work).  Tiles of one bucket come in no fixed order.
constexpr int kOrderBuckets = 4096;
constexpr int kOrderChunk = 8;  // tiles whose work one thread loads at once
struct TileOrderShared {
    uint32_t cnt[kOrderBuckets];
    uint32_t wave_tot[16];
};

// Buckets of the tiles t0 + c NT, c < kOrderChunk: the loads go out
// together (indices clamped to the last tile, so none is predicated away),
// then tiles past ntiles are marked with kOrderBuckets.
template <int NT>
__device__ __forceinline__ void order_buckets(const uint2 *ranges, const uint32_t *work, uint32_t ntiles,
                                              uint32_t t0, uint32_t bk[kOrderChunk]) {
    uint32_t wk[kOrderChunk];
    if (work) {
#pragma unroll
        for (int c = 0; c < kOrderChunk; ++c) wk[c] = work[min(t0 + (uint32_t)(c * NT), ntiles - 1u)];
    } else {
        uint2 r[kOrderChunk];
#pragma unroll
        for (int c = 0; c < kOrderChunk; ++c) r[c] = ranges[min(t0 + (uint32_t)(c * NT), ntiles - 1u)];
#pragma unroll
        for (int c = 0; c < kOrderChunk; ++c) wk[c] = r[c].y - r[c].x;
    }
#pragma unroll
    for (int c = 0; c < kOrderChunk; ++c)
        bk[c] = t0 + (uint32_t)(c * NT) < ntiles
                    ? (uint32_t)(kOrderBuckets - 1) - min(wk[c], (uint32_t)(kOrderBuckets - 1))
                    : (uint32_t)kOrderBuckets;
}

// The order, written by the NT threads of the calling workgroup (all of
// them call it; ntiles > 0).
template <int NT>
__device__ inline void tile_order_block(const uint2 *ranges, const uint32_t *work, uint32_t ntiles, uint32_t *order,
                                        TileOrderShared &sh) {
    static_assert(NT % kWave == 0 && NT / kWave <= 16 && kOrderBuckets % NT == 0, "workgroup shape");
    for (int b = threadIdx.x; b < kOrderBuckets; b += NT) sh.cnt[b] = 0;
    __syncthreads();
    for (uint32_t t0 = threadIdx.x; t0 < ntiles; t0 += NT * kOrderChunk) {
        uint32_t bk[kOrderChunk];
        order_buckets<NT>(ranges, work, ntiles, t0, bk);
#pragma unroll
        for (int c = 0; c < kOrderChunk; ++c)
            if (bk[c] < kOrderBuckets) atomicAdd(&sh.cnt[bk[c]], 1u);
    }
    __syncthreads();
    // exclusive scan of the bucket counts: kPer per thread, then across waves
    constexpr int kPer = kOrderBuckets / NT;
    uint32_t v[kPer], sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        v[k] = sh.cnt[threadIdx.x * kPer + k];
        sum += v[k];
    }
    const int lane = __lane_id(), wv = threadIdx.x / kWave;
    uint32_t x = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) sh.wave_tot[wv] = x;
    __syncthreads();
    uint32_t run = x - sum;
    for (int k = 0; k < wv; ++k) run += sh.wave_tot[k];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        sh.cnt[threadIdx.x * kPer + k] = run;
        run += v[k];
    }
    __syncthreads();
    for (uint32_t t0 = threadIdx.x; t0 < ntiles; t0 += NT * kOrderChunk) {
        uint32_t bk[kOrderChunk];
        order_buckets<NT>(ranges, work, ntiles, t0, bk);
#pragma unroll
        for (int c = 0; c < kOrderChunk; ++c)
            if (bk[c] < kOrderBuckets) order[atomicAdd(&sh.cnt[bk[c]], 1u)] = t0 + (uint32_t)(c * NT);
    }
}

// Optimisation (optim.hip).  Parameter arrays as five segments.
constexpr int kSegments = 5;
enum { kSegMeans = 0, kSegLogScales = 1, kSegQuats = 2, kSegLogits = 3, kSegSh = 4 };
struct OptimArrays {
    float *ptr[kSegments];
};
struct AdamArgs {
    int64_t total;               // elements in all segments
    int64_t begin[kSegments];    // first element of each segment
    float lr[kSegments];         // per segment (the SH segment's: degree 0)
    float lr_sh_rest;            // SH degrees >= 1
    int64_t sh_stride;           // floats of SH per Gaussian
    float beta1, beta2, eps, inv_bc1, inv_sqrt_bc2;
};
struct DensifyArgs {
    float tau, log_clone, logit_min, max_screen, log_big, log_shrink;
    int screen_on;
};
// skip (device, may be null): nothing is written when *skip != 0.
hipError_t launch_adam(const OptimArrays &P, const OptimArrays &G, const OptimArrays &M1, const OptimArrays &M2,
                       const AdamArgs &a, float *act_scales, float *act_opacities, const int32_t *skip,
                       hipStream_t st);
hipError_t launch_stats(const uint32_t *n_tiles, const float *radii, const float *dscreen, int64_t n, float *accum,
                        float *denom, float *max_radius, const int32_t *skip, hipStream_t st);
hipError_t launch_dens_flags(const OptimArrays &P, const float *accum, const float *denom, const float *max_radius,
                             int64_t n, const DensifyArgs &d, uint32_t *flags, hipStream_t st);
hipError_t launch_dens_scatter(const OptimArrays &P, const OptimArrays &M1, const OptimArrays &M2,
                               const uint32_t *flags, const uint32_t *pos, const float *noise, int64_t n,
                               int sh_floats, float log_shrink, const OptimArrays &PO, const OptimArrays &M1O,
                               const OptimArrays &M2O, hipStream_t st);
hipError_t launch_reset_opacity(float *logits, float *m1, float *m2, int64_t n, float lo, hipStream_t st);

// Photometric loss (1 - lambda) L1 + lambda (1 - SSIM) of [channels][H][W]
// images, weighted by the [H][W] mask (may be null), and its gradient (grad
// may be null); scratch from ssim_scratch_bytes (with_grad: room for the
// three filtered planes).
size_t ssim_scratch_bytes(int channels, int height, int width, bool with_grad);
hipError_t launch_photometric(const float *image, const float *target, const float *mask, int channels, int height,
                              int width, float lambda, float *grad, float *loss, void *scratch, hipStream_t st);

// L1 loss.
// Ceilings: FMA, exp2, scattered-atomic and copy kernels, each timed with
// HIP events over `repeats` launches after a warm-up; ms[k] per launch and
// work[k] per launch (FLOP, exp2 results, atomics, bytes moved).  A null
// atomic buffer or copy source skips that measurement (ms = work = 0).
hipError_t measure_ceilings(float *atomic_buf, uint32_t atomic_words, const float *copy_src, float *copy_dst,
                            int64_t copy_bytes, int repeats, double ms[4], double work[4], hipStream_t st);

size_t l1_scratch_bytes();
hipError_t launch_l1(const float *image, const float *target, int64_t count, float *grad, float *loss,
                     void *scratch, hipStream_t st);

}  // namespace omnigs
