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
    float px_hi, px_lo, py_hi, py_lo;  // ERP pixel position of the centre (Eq. 5)
    float q00, q01, q11, opacity;      // inverse 2D covariance (Eq. 8), opacity
    float r, g, b;                     // SH colour, clamped at 0
    float reach;                       // log2(opacity / alpha_min): alpha >= alpha_min
                                       // iff -log2(e)/2 d^T Q d >= -reach
};
static_assert(sizeof(BlendRecord) == 48, "record layout");

// Per-Gaussian screen-space gradient accumulators written by the backward
// blend: dL/dp (2), dL/dQ (q00, q01, q11), dL/do, dL/drgb (3).
constexpr int kAcc = 9;

// Depth-sort key of a culled Gaussian: sorts after every finite t_r.
constexpr uint32_t kCulledKey = 0xffffffffu;

struct ProjectArgs {
    const float *means, *scales, *quats, *opacities, *sh;
    int64_t n;
    int sh_degree, sh_coeffs;
    double R[9], t[3], campos[3];
    int width, height, tiles_x, tiles_y;
    double alpha_min, dilation, near_plane;
};

struct FrameGeom {  // one camera's image inside a (possibly batched) launch
    int width, height, tiles_x, tiles_y;
    uint32_t tile_base;  // first global tile id of this image
};

// Camera-dependent part of ProjectArgs, one entry per camera of a batch.
struct CamGeom {
    double R[9], t[3], campos[3];
    int width, height, tiles_x, tiles_y;
};
struct CamTable {
    int count;
    CamGeom c[kMaxBatch];
};

// Tile geometry of the cameras behind record index g = b * n_per + i.
struct EmitFrames {
    int64_t n_per;  // records per camera
    int count;
    int tiles_x[kMaxBatch];
    uint32_t tile_base[kMaxBatch];
};

// Host-side launchers (each .hip file owns its kernels).
hipError_t launch_project(const ProjectArgs &a, BlendRecord *rec, uint32_t *depth_key, uint32_t *n_tiles,
                          uint2 *rect, hipStream_t st);
// All cameras of `cams` in one launch: the outputs of camera b for Gaussian i
// land at index b * a.n + i, bit-identical to launch_project of that camera
// (a's camera fields are ignored).
hipError_t launch_project_batch(const ProjectArgs &a, const CamTable &cams, BlendRecord *rec, uint32_t *depth_key,
                                uint32_t *n_tiles, uint2 *rect, hipStream_t st);
hipError_t launch_project_backward(const ProjectArgs &a, const uint32_t *n_tiles, const float *acc,
                                   const omnigs_grads &gr, hipStream_t st);

// radix sort of (u32 key, u32 value) pairs on the low `bits` bits of the key;
// stable.  Result lands in keys_out/vals_out.  `scratch` from sort_scratch_bytes.
// n_dev (device, may be null): the element count is min(n, *n_dev), read on
// the device (n then only bounds the buffers and the grid).
size_t sort_scratch_bytes(int64_t n);
hipError_t radix_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_tmp,
                            uint32_t *vals_tmp, uint32_t *keys_out, uint32_t *vals_out, int64_t n, int bits,
                            void *scratch, hipStream_t st, const uint32_t *n_dev = nullptr);
hipError_t launch_iota(uint32_t *v, int64_t n, hipStream_t st);

// Exclusive scan of u32 (optionally of in[gather[i]]); *total (device, may be
// null) receives the sum.  `scratch` from scan_scratch_bytes.
size_t scan_scratch_bytes(int64_t n);
hipError_t scan_exclusive(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total, void *scratch,
                          hipStream_t st, const uint32_t *gather);

// Instance emission in depth order: offs[r] = exclusive scan of the tile
// counts in depth order (offs[n] = M at *m_dev).  Writes min(M, capacity)
// instances, with global tile ids (frames.tile_base of the record's camera
// plus the tile inside its image); sets *overflow when M > capacity.  `part`
// holds emit_blocks(capacity) entries of scratch.
uint64_t emit_blocks(uint64_t capacity);
hipError_t launch_emit(const uint32_t *order, const uint32_t *n_tiles, const uint2 *rect, const uint32_t *offs,
                       int64_t n, uint32_t *part, const uint32_t *m_dev, const EmitFrames &frames,
                       uint64_t capacity, uint32_t *inst_tile, uint32_t *inst_gauss, int32_t *overflow,
                       hipStream_t st);
hipError_t launch_tile_ranges(const uint32_t *inst_tile, const uint32_t *m_dev, uint64_t capacity,
                              uint2 *ranges, uint32_t n_tiles_total, hipStream_t st);

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);

// Blend kernels.
struct BlendSettings {
    float alpha_min, alpha_max, T_min;
    float bg[3];
};
// `order` (device, may be null): launch order of the tiles (a permutation).
// The forward writes each tile's largest contributor count (the backward's
// walk length) to tile_work (may be null).
hipError_t launch_blend_forward(const FrameGeom &f, const BlendRecord *rec, const uint32_t *inst_gauss,
                                const uint2 *ranges, const BlendSettings &s, float *image, float *final_T,
                                int32_t *n_contrib, int32_t *n_blended, const uint32_t *order, uint32_t *tile_work,
                                hipStream_t st);
// Forward blend of several images in one launch over their concatenated
// tile space (frames[k].tile_base ascending, total_tiles in all).
hipError_t launch_blend_forward_frames(const FrameGeom *frames, const omnigs_image_out *outs, int count,
                                       const BlendRecord *rec, const uint32_t *inst_gauss, const uint2 *ranges,
                                       const BlendSettings &s, const uint32_t *order, uint32_t total_tiles,
                                       hipStream_t st);
hipError_t launch_blend_backward(const FrameGeom &f, const BlendRecord *rec, const uint32_t *inst_gauss,
                                 const uint2 *ranges, const BlendSettings &s, const float *final_T,
                                 const int32_t *n_contrib, const float *dL_dimage, float *acc, const uint32_t *order,
                                 hipStream_t st);
// Longest-first tile order from the list lengths (work == null) or from a
// per-tile work array.  One workgroup; ntiles unbounded.
hipError_t launch_tile_order(const uint2 *ranges, const uint32_t *work, uint32_t ntiles, uint32_t *order,
                             hipStream_t st);

// L1 loss.
size_t l1_scratch_bytes();
hipError_t launch_l1(const float *image, const float *target, int64_t count, float *grad, float *loss,
                     void *scratch, hipStream_t st);

}  // namespace omnigs
