// capi.hip -- the extern "C" entry points of libomnigs.so (include/omnigs.h):
// argument validation, carving of caller-allocated device memory, stage
// sequencing on the caller's stream, optional per-stage HIP-event timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

using namespace omnigs;

namespace {

thread_local std::string g_error;

omnigs_status fail(omnigs_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                                   \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess) return fail(OMNIGS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

// ------------------------------------------------------------- stage timing
enum Stage {
    kStProject = 0,
    kStDepthSort,
    kStEmitCount,
    kStSuperEmit,
    kStSuperSort,
    kStTileBin,
    kStTileOrder,  // records nothing: the forward's tile order is written inside the
                   // tile binning, the backward's with the accumulator clear (the
                   // stage keeps its index so that callers' stage masks stay valid)
    kStBlendFwd,
    kStL1,
    kStBwdClear,
    kStBlendBwd,
    kStProjectBwd,
    kStStats,
    kStAdam,
    kStDensify,
    kStCount
};
const char *kStageNames[kStCount] = {"project",    "depth_sort", "emit_count", "super_emit", "super_sort",
                                     "tile_bin",   "tile_order", "blend_fwd",  "l1_loss",    "bwd_clear",
                                     "blend_bwd",  "project_bwd", "stats",      "adam",       "densify"};

struct Profiler {
    std::mutex mu;
    std::atomic<uint32_t> stages{0};  // bit k: stage k is timed (read without the lock)
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    double ms[kStCount] = {};
    int64_t launches[kStCount] = {};

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};
Profiler g_prof;

// Brackets one stage with events on the stream when profiling is enabled.
struct StageTimer {
    hipStream_t st;
    int stage;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(hipStream_t s, int stg) : st(s), stage(stg) {
        if (!((g_prof.stages.load(std::memory_order_relaxed) >> stg) & 1u)) return;
        std::lock_guard<std::mutex> lk(g_prof.mu);
        a = g_prof.get();
        b = g_prof.get();
        if (a) (void)hipEventRecord(a, st);
    }
    ~StageTimer() {
        if (!a || !b) return;
        (void)hipEventRecord(b, st);
        std::lock_guard<std::mutex> lk(g_prof.mu);
        g_prof.pending.push_back({stage, a, b});
    }
};

// ------------------------------------------------------------ memory arenas
constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// Two-phase carving: the first pass (base == nullptr) measures, the second
// hands out 256-byte aligned sub-buffers of one allocation.
struct Arena {
    char *base = nullptr;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        off = align_up(off);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    void *take_bytes(size_t bytes) { return take<char>(bytes); }
};

omnigs_status alloc_arena(omnigs_allocator A, size_t bytes, int32_t kind, Arena &ar, const char *what) {
    ar.off = 0;
    if (bytes == 0) bytes = kAlign;
    void *p = A.alloc(A.user, align_up(bytes), kind);
    if (!p) return fail(OMNIGS_ERR_ALLOC, "allocator returned NULL for %s (%zu bytes)", what, bytes);
    if (reinterpret_cast<uintptr_t>(p) % 16 != 0)
        return fail(OMNIGS_ERR_ALLOC, "allocator returned a pointer not 16-byte aligned for %s", what);
    ar.base = static_cast<char *>(p);
    return OMNIGS_OK;
}

// ---------------------------------------------------------------- validation
omnigs_status check_gaussians(const omnigs_gaussians *g) {
    if (!g) return fail(OMNIGS_ERR_INVALID, "gaussians is NULL");
    if (g->n < 0 || g->n >= (int64_t(1) << 31)) return fail(OMNIGS_ERR_INVALID, "n = %lld out of range", (long long)g->n);
    if (g->sh_degree < 0 || g->sh_degree > 3) return fail(OMNIGS_ERR_INVALID, "sh_degree %d not in 0..3", g->sh_degree);
    const int need = (g->sh_degree + 1) * (g->sh_degree + 1);
    if (g->sh_coeffs < need || g->sh_coeffs > 16)
        return fail(OMNIGS_ERR_INVALID, "sh_coeffs %d not in [%d, 16]", g->sh_coeffs, need);
    if (g->n > 0 && (!g->means || !g->scales || !g->quats || !g->opacities || !g->sh))
        return fail(OMNIGS_ERR_INVALID, "a Gaussian parameter pointer is NULL");
    if (g->n > 0 && reinterpret_cast<uintptr_t>(g->quats) % 16 != 0)
        return fail(OMNIGS_ERR_INVALID, "quats must be 16-byte aligned");
    return OMNIGS_OK;
}

omnigs_status check_camera(const omnigs_camera *c) {
    if (!c) return fail(OMNIGS_ERR_INVALID, "camera is NULL");
    if (c->model != OMNIGS_CAMERA_ERP && c->model != OMNIGS_CAMERA_PINHOLE)
        return fail(OMNIGS_ERR_INVALID, "unknown camera model %d", c->model);
    if (c->rows < 0 || c->rows > c->height)
        return fail(OMNIGS_ERR_INVALID, "rows %d not in [0, height %d]", c->rows, c->height);
    if (c->model == OMNIGS_CAMERA_ERP && (c->width <= 0 || c->width % kTile != 0 || c->width > 65520))
        return fail(OMNIGS_ERR_INVALID, "ERP width %d must be a positive multiple of 16, <= 65520", c->width);
    if (c->model == OMNIGS_CAMERA_PINHOLE) {
        if (c->width < 1 || c->width > 65520) return fail(OMNIGS_ERR_INVALID, "width %d not in [1, 65520]", c->width);
        if (!(c->fx > 0.0) || !(c->fy > 0.0) || !std::isfinite(c->fx) || !std::isfinite(c->fy) ||
            !std::isfinite(c->cx) || !std::isfinite(c->cy))
            return fail(OMNIGS_ERR_INVALID, "pinhole intrinsics need finite fx, fy > 0 and finite cx, cy");
    }
    if (c->height < 1 || c->height > 65520) return fail(OMNIGS_ERR_INVALID, "height %d not in [1, 65520]", c->height);
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(c->R_cw[k])) return fail(OMNIGS_ERR_INVALID, "non-finite camera rotation");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(c->t_cw[k])) return fail(OMNIGS_ERR_INVALID, "non-finite camera translation");
    return OMNIGS_OK;
}

omnigs_status check_settings(const omnigs_settings *s) {
    if (!s) return fail(OMNIGS_ERR_INVALID, "settings is NULL");
    if (!(s->alpha_min > 0.0 && s->alpha_min < 1.0)) return fail(OMNIGS_ERR_INVALID, "alpha_min must be in (0, 1)");
    if (!(s->alpha_max >= s->alpha_min && s->alpha_max < 1.0))
        return fail(OMNIGS_ERR_INVALID, "alpha_max must be in [alpha_min, 1)");
    if (!(s->T_min > 0.0 && s->T_min < 1.0) || !((float)s->T_min > 0.0f))
        return fail(OMNIGS_ERR_INVALID, "T_min must be in (0, 1) and positive as a float");
    if (!(s->dilation >= 0.0) || !std::isfinite(s->dilation)) return fail(OMNIGS_ERR_INVALID, "bad dilation");
    if (!(s->near_plane >= 0.0) || !std::isfinite(s->near_plane)) return fail(OMNIGS_ERR_INVALID, "bad near_plane");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(s->bg[k])) return fail(OMNIGS_ERR_INVALID, "non-finite background");
    return OMNIGS_OK;
}

ProjectArgs make_project_args(const omnigs_gaussians *g, const omnigs_camera *c, const omnigs_settings *s) {
    ProjectArgs a{};
    a.means = g->means;
    a.scales = g->scales;
    a.quats = g->quats;
    a.opacities = g->opacities;
    a.sh = g->sh;
    a.n = g->n;
    a.sh_degree = g->sh_degree;
    a.sh_coeffs = g->sh_coeffs;
    for (int k = 0; k < 9; ++k) a.R[k] = c->R_cw[k];
    for (int k = 0; k < 3; ++k) a.t[k] = c->t_cw[k];
    // camera centre in world coordinates: -R^T t
    for (int k = 0; k < 3; ++k) a.campos[k] = -(c->R_cw[k] * c->t_cw[0] + c->R_cw[3 + k] * c->t_cw[1] + c->R_cw[6 + k] * c->t_cw[2]);
    a.width = c->width;
    a.height = c->height;
    a.model = c->model;
    a.fx = c->fx;
    a.fy = c->fy;
    a.cx = c->cx;
    a.cy = c->cy;
    // the ERP width is a multiple of the tile; a pinhole image may end in a
    // partial tile column
    a.tiles_x = (c->width + kTile - 1) / kTile;
    a.rows = c->rows > 0 ? c->rows : c->height;  // the image holds the top `rows` rows
    a.tiles_y = (a.rows + kTile - 1) / kTile;
    a.alpha_min = s->alpha_min;
    a.dilation = s->dilation;
    a.near_plane = s->near_plane;
    return a;
}

BlendSettings make_blend_settings(const omnigs_settings *s) {
    BlendSettings b{};
    b.alpha_min = (float)s->alpha_min;
    b.alpha_max = (float)s->alpha_max;
    b.T_min = (float)s->T_min;
    for (int k = 0; k < 3; ++k) b.bg[k] = (float)s->bg[k];
    return b;
}

int bits_for(uint64_t count) {
    int b = 1;
    while (b < 32 && (uint64_t(1) << b) < count) ++b;
    return b;
}

// Per-record buffers of one forward: persistent part (state) and scratch.
struct GeomState {
    BlendRecord *rec;
    uint32_t *n_tiles, *order;
    uint2 *rect;
    float *radii, *depth;
    uint32_t *totals;  // [0] super entries S, [1] tile instances M (adjacent: one readback),
                       // [2] fault bits (bit 0: a lookback wait gave up)
    void carve(Arena &a, int64_t n) {
        const size_t m = (size_t)(n > 0 ? n : 1);
        rec = a.take<BlendRecord>(m);
        n_tiles = a.take<uint32_t>(m);
        order = a.take<uint32_t>(m);
        rect = a.take<uint2>(m);
        radii = a.take<float>(m);
        depth = a.take<float>(m);
        totals = a.take<uint32_t>(3);
    }
};
struct GeomScratch {
    uint32_t *depth_key, *keys_tmp, *vals_tmp, *keys_sorted, *offs, *n_super;
    void *sort_tmp, *scan_tmp;
    void carve(Arena &a, int64_t n) {
        const size_t m = (size_t)(n > 0 ? n : 1);
        depth_key = a.take<uint32_t>(m);
        keys_tmp = a.take<uint32_t>(m);
        vals_tmp = a.take<uint32_t>(m);
        keys_sorted = a.take<uint32_t>(m);
        offs = a.take<uint32_t>(m + 1);
        n_super = a.take<uint32_t>(m);
        sort_tmp = a.take_bytes(sort_scratch_bytes((int64_t)m));
        scan_tmp = a.take_bytes(scan_scratch_bytes((int64_t)m));
    }
};

// Depth sort and per-rank super-entry offsets of n records (projected
// already, which left M = total tile instances at gst.totals[1]): gs.offs
// and S at gst.totals[0].
// cleared: the sort's and the scan's lookback words are already zero
// (geom_clear).
// part: when given, the scan also writes the emission's partition.
omnigs_status sort_and_count(int64_t n, GeomState &gst, GeomScratch &gs, hipStream_t st, bool cleared = false,
                             ScanPartition part = {}) {
    {
        StageTimer t(st, kStDepthSort);
        HIP_TRY(radix_sort_pairs(gs.depth_key, nullptr, gs.keys_tmp, gs.vals_tmp, gs.keys_sorted, gst.order, n, 32,
                                 gs.sort_tmp, st, nullptr, nullptr, 0, cleared, gst.totals + 2));
    }
    {
        StageTimer t(st, kStEmitCount);
        HIP_TRY(scan_exclusive(gs.n_super, gs.offs, n, gst.totals, gs.scan_tmp, st, gst.order, cleared,
                               gst.totals + 2, part));
    }
    return OMNIGS_OK;
}

// The words that sort_and_count with cleared == true expects zero, and the
// counters of the state.
void geom_clear(int64_t n, GeomState &gst, GeomScratch &gs, ClearList &L) {
    const int64_t m = n > 0 ? n : 1;
    L.add(gs.sort_tmp, sort_clear_words(m, 32));
    L.add(gs.scan_tmp, scan_clear_words(m));
    L.add(gst.totals, 3);
}

// Largest block count of a launch whose block-entry keys carry the covers
// (omnigs_set_cover_key_blocks lowers it to test the other path).
uint32_t g_cover_key_blocks = kMaxCoverKeyBlocks;

// Grids of the images of a launch.
struct Grids {
    EmitFrames ef{};   // super-tile emission
    SuperTable sup{};  // super-tile and tile grids
    uint32_t n_super = 0, n_tiles = 0;
    void add(int b, int tiles_x, int tiles_y) {
        const int sx = (tiles_x + kSuper - 1) / kSuper, sy = (tiles_y + kSuper - 1) / kSuper;
        ef.tiles_x[b] = tiles_x;
        ef.cols[b] = sx;
        ef.base[b] = n_super;
        sup.f[b] = SuperFrame{n_super, n_tiles, sx, sy, tiles_x, tiles_y};
        n_super += (uint32_t)(sx * sy);
        n_tiles += (uint32_t)(tiles_x * tiles_y);
        ef.cover_key = n_super <= g_cover_key_blocks;
    }
};

// Scratch of the two-level binning for super_cap super entries.
struct BinScratch {
    uint32_t *stile, *sgauss, *stile_tmp, *sgauss_tmp, *part;
    uint2 *sranges;
    void *sort_tmp, *bin_tmp;
    void carve(Arena &a, uint64_t super_cap, uint32_t n_super) {
        const size_t m = (size_t)(super_cap > 0 ? super_cap : 1);
        stile = a.take<uint32_t>(m);
        sgauss = a.take<uint32_t>(m);
        stile_tmp = a.take<uint32_t>(m);
        sgauss_tmp = a.take<uint32_t>(m);
        part = a.take<uint32_t>((size_t)emit_blocks(super_cap) + 1);
        sranges = a.take<uint2>(n_super > 0 ? n_super : 1);
        sort_tmp = a.take_bytes(sort_scratch_bytes((int64_t)m));
        bin_tmp = a.take_bytes(binning_scratch_bytes(super_cap, n_super));
    }
};

// Two-level binning of nrec depth-sorted records into per-tile lists:
// super-tile entries in depth order (emission), a stable sort by super-tile,
// and the expansion into the lists of the tiles (bin.hip).  With counted ==
// true the entry count is read on the device (min(S, super_cap)).
omnigs_status run_binning(int64_t nrec, const GeomState &gst, const GeomScratch &gs, const Grids &G,
                          uint64_t super_cap, uint64_t inst_cap, bool counted, BinScratch &bs, uint2 *ranges,
                          uint32_t *inst_gauss, int32_t *overflow, hipStream_t st, bool cleared = false,
                          uint32_t *order = nullptr, uint32_t order_tiles = 0, bool partitioned = false) {
    const int bits = bits_for(G.n_super);
    const bool odd = ((bits + 7) / 8) % 2;
    uint32_t *et = odd ? bs.stile_tmp : bs.stile, *eg = odd ? bs.sgauss_tmp : bs.sgauss;
    {
        StageTimer t(st, kStSuperEmit);
        // emit where the sort's ping-pong starts, so that the last pass lands
        // in stile / sgauss
        HIP_TRY(launch_emit(gst.order, gst.rect, gs.offs, nrec, bs.part, gst.totals, G.ef, super_cap, et, eg, overflow,
                            st, partitioned));
    }
    {
        StageTimer t(st, kStSuperSort);
        // one pass (up to 256 blocks): the sort writes each block's range
        // from its digit totals; else the ranges from adjacent sorted keys
        const bool one_pass = bits <= 8;
        HIP_TRY(radix_sort_pairs(et, eg, bs.stile_tmp, bs.sgauss_tmp, bs.stile, bs.sgauss, (int64_t)super_cap, bits,
                                 bs.sort_tmp, st, counted ? gst.totals : nullptr, one_pass ? bs.sranges : nullptr,
                                 one_pass ? (int)G.n_super : 0, cleared, gst.totals + 2));
        if (!one_pass) {
            HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(bs.sranges), 0u, 2 * (int64_t)G.n_super, st));
            HIP_TRY(launch_tile_ranges(bs.stile, gst.totals, super_cap, bs.sranges, G.n_super,
                                       G.ef.cover_key ? kMaxCoverKeyBlocks - 1u : ~0u, st));
        }
    }
    {
        StageTimer t(st, kStTileBin);
        HIP_TRY(launch_binning(G.sup, G.n_super, gst.rect, G.ef.cover_key ? bs.stile : nullptr, bs.sgauss, bs.sranges,
                               super_cap, inst_cap, bs.bin_tmp,
                               ranges, inst_gauss, overflow, st, cleared, gst.totals + 2, order, order_tiles));
    }
    return OMNIGS_OK;
}

}  // namespace

// The words that run_binning with cleared == true expects zero.
void bin_clear(uint64_t super_cap, const Grids &G, BinScratch &bs, ClearList &L) {
    L.add(bs.sort_tmp, sort_clear_words((int64_t)(super_cap > 0 ? super_cap : 1), bits_for(G.n_super)));
    binning_clear(bs.bin_tmp, super_cap, G.n_super, L);
}

// Device scratch of omnigs_backward_noalloc (gradient accumulators and the
// tile launch order of one backward), for callers that cannot allocate.
// Every device the library runs on holds its own copy until the process
// ends; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's name in host code
// is a host-side stand-in, not a device address).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
char *g_noalloc_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up once per device.
omnigs_status noalloc_scratch(char *&base) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(OMNIGS_ERR_INVALID, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(OMNIGS_ERR_HIP, "hipGetSymbolAddress returned NULL for the no-alloc scratch");
        g_noalloc_ptr[dev] = static_cast<char *>(p);
    }
    base = g_noalloc_ptr[dev];
    return OMNIGS_OK;
}

// The checks and stages of the backward on caller-provided scratch: `carve`
// maps the accumulator and tile-order sizes to their buffers (or fails).
template <class Carve>
omnigs_status backward_impl(const omnigs_gaussians *g, const omnigs_camera *cam, const omnigs_settings *s,
                            const omnigs_state *state, const omnigs_image_out *fwd, const float *dL_dimage,
                            const float *dL_ddepth, const float *dL_dalpha, omnigs_grads *grads, void *stream,
                            Carve carve) {
    omnigs_status rc;
    if ((rc = check_gaussians(g)) != OMNIGS_OK) return rc;
    if ((rc = check_camera(cam)) != OMNIGS_OK) return rc;
    if ((rc = check_settings(s)) != OMNIGS_OK) return rc;
    if (!state || !fwd || !fwd->final_T || !fwd->n_contrib || !dL_dimage || !grads)
        return fail(OMNIGS_ERR_INVALID, "a state, forward-output, cotangent or gradient pointer is NULL");
    if (g->n > 0 && (!grads->dmeans || !grads->dscales || !grads->dquats || !grads->dopacities || !grads->dsh ||
                     !grads->dscreen))
        return fail(OMNIGS_ERR_INVALID, "a gradient output pointer is NULL");
    if (g->n > 0 && reinterpret_cast<uintptr_t>(grads->dquats) % 16 != 0)
        return fail(OMNIGS_ERR_INVALID, "dquats must be 16-byte aligned");
    const bool aux = dL_ddepth || dL_dalpha;
    if (state->n != g->n || state->width != cam->width ||
        state->height != (cam->rows > 0 ? cam->rows : cam->height))
        return fail(OMNIGS_ERR_INVALID, "state does not match the Gaussians / camera");
    if (aux && g->n > 0 && !state->depth) return fail(OMNIGS_ERR_INVALID, "state depth buffer is NULL");
    if (g->n > 0 && (!state->records || !state->n_tiles || !state->inst_gauss || !state->tile_range ||
                     !state->tile_work))
        return fail(OMNIGS_ERR_INVALID, "state buffers are NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = g->n;
    if (n == 0) return OMNIGS_OK;
    const ProjectArgs pa = make_project_args(g, cam, s);
    const uint32_t ntiles = (uint32_t)(pa.tiles_x * pa.tiles_y);
    const int nacc = aux ? kAccAux : kAcc;  // accumulator fields per Gaussian
    float *acc = nullptr;
    uint32_t *order = nullptr;
    if ((rc = carve((size_t)n * nacc, (size_t)ntiles, acc, order)) != OMNIGS_OK) return rc;
    const auto *rec = static_cast<const BlendRecord *>(state->records);
    const auto *ranges = reinterpret_cast<const uint2 *>(state->tile_range);
    {
        // the accumulators cleared and the tile order (longest recorded walk
        // first) in one launch
        StageTimer t(st, kStBwdClear);
        HIP_TRY(launch_clear_and_order(reinterpret_cast<uint32_t *>(acc), n * nacc, state->tile_work, ntiles, order,
                                       st));
    }
    const FrameGeom f{cam->width, pa.rows, pa.tiles_x, pa.tiles_y, 0u, pa.model == OMNIGS_CAMERA_ERP};
    {
        StageTimer t(st, kStBlendBwd);
        HIP_TRY(launch_blend_backward(f, rec, state->depth, state->inst_gauss, ranges, make_blend_settings(s),
                                      fwd->final_T, fwd->n_contrib, dL_dimage, dL_ddepth, dL_dalpha, acc, order, st, state->inst_quad));
    }
    {
        StageTimer t(st, kStProjectBwd);
        HIP_TRY(launch_project_backward(pa, state->n_tiles, acc, nacc, *grads, st));
    }
    return OMNIGS_OK;
}

// Buffers of omnigs_forward_batch.  Its allocations and the size query
// omnigs_forward_batch_bytes run the same carving (a measuring pass on a
// null arena gives the byte count that the allocator is asked for).
struct BatchBuffers {
    GeomState gst;
    GeomScratch gs;
    uint32_t *inst_gauss = nullptr, *order = nullptr;
    uint2 *ranges = nullptr;
    BinScratch bs;
    void carve_records(Arena &a, int64_t nrec) {
        gst.carve(a, nrec);
        gs.carve(a, nrec);
    }
    void carve_instances(Arena &a, uint64_t inst_cap, uint64_t super_cap, uint32_t ntiles, const Grids &G) {
        inst_gauss = a.take<uint32_t>((size_t)(inst_cap > 0 ? inst_cap : 1));
        ranges = a.take<uint2>(ntiles);
        order = a.take<uint32_t>(ntiles);
        bs.carve(a, super_cap, G.n_super);
    }
};

// The bytes alloc_arena requests for an arena of `off` measured bytes.
size_t arena_request(size_t off) { return align_up(off == 0 ? kAlign : off); }

// Camera checks and the grids of a batch: tiles per frame, stacked.
omnigs_status batch_grids(const omnigs_camera *cams, int32_t batch, int64_t n, Grids &G, uint64_t &total_tiles) {
    if (batch < 1 || batch > kMaxBatch) return fail(OMNIGS_ERR_INVALID, "batch %d not in [1, %d]", batch, kMaxBatch);
    if (!cams) return fail(OMNIGS_ERR_INVALID, "cameras is NULL");
    G = Grids{};
    G.ef.n_per = n > 0 ? n : 1;
    G.ef.count = batch;
    G.ef.super = 1;
    G.sup.count = batch;
    total_tiles = 0;
    omnigs_status rc;
    for (int b = 0; b < batch; ++b) {
        if ((rc = check_camera(&cams[b])) != OMNIGS_OK) return rc;
        const int tiles_x = (cams[b].width + kTile - 1) / kTile;
        const int rows = cams[b].rows > 0 ? cams[b].rows : cams[b].height;
        const int tiles_y = (rows + kTile - 1) / kTile;
        total_tiles += (uint64_t)tiles_x * tiles_y;
        if (total_tiles >= (uint64_t(1) << 31)) return fail(OMNIGS_ERR_INVALID, "too many tiles in the batch");
        G.add(b, tiles_x, tiles_y);
    }
    return OMNIGS_OK;
}

}  // namespace

// ============================================================== public API
extern "C" {

omnigs_settings omnigs_default_settings(void) {
    omnigs_settings s;
    s.alpha_min = 1.0 / 255.0;
    s.alpha_max = 0.99;
    s.T_min = 1e-4;
    s.dilation = 0.3;
    s.near_plane = 0.2;
    s.bg[0] = s.bg[1] = s.bg[2] = 0.0;
    return s;
}

const char *omnigs_last_error(void) { return g_error.c_str(); }

omnigs_status omnigs_forward(const omnigs_gaussians *g, const omnigs_camera *cam, const omnigs_settings *s,
                             omnigs_allocator alloc, omnigs_image_out *out, omnigs_state *state,
                             const omnigs_capacity *cap, void *stream) {
    omnigs_status rc;
    if ((rc = check_gaussians(g)) != OMNIGS_OK) return rc;
    if ((rc = check_camera(cam)) != OMNIGS_OK) return rc;
    if ((rc = check_settings(s)) != OMNIGS_OK) return rc;
    if (!alloc.alloc) return fail(OMNIGS_ERR_INVALID, "allocator callback is NULL");
    if (!out || !out->image || !out->final_T || !out->n_contrib) return fail(OMNIGS_ERR_INVALID, "output pointer is NULL");
    if (!state) return fail(OMNIGS_ERR_INVALID, "state is NULL");
    const bool counted = cap && cap->instances > 0;
    if (cap) {
        const int64_t lim = (int64_t(1) << 31) - 1;
        if (cap->instances < 0 || cap->instances >= lim || cap->entries < 0 || cap->entries >= lim)
            return fail(OMNIGS_ERR_INVALID, "capacities (%lld instances, %lld entries) out of range",
                        (long long)cap->instances, (long long)cap->entries);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const ProjectArgs pa = make_project_args(g, cam, s);
    const int64_t n = g->n;
    const uint32_t ntiles = (uint32_t)(pa.tiles_x * pa.tiles_y);

    Grids G;
    G.ef.n_per = n > 0 ? n : 1;
    G.ef.count = 1;
    G.ef.super = 1;
    G.sup.count = 1;
    G.add(0, pa.tiles_x, pa.tiles_y);
    // N-sized state and scratch; M-sized state and S-sized scratch, with the
    // caller's capacities (allocated with the N-sized buffers) or the counts
    // read back after the depth sort
    GeomState gst;
    GeomScratch gs;
    uint64_t super_cap = 0, inst_cap = 0;
    uint32_t *inst_gauss = nullptr, *tile_work = nullptr, *order = nullptr;
    uint8_t *inst_quad = nullptr;
    uint2 *ranges = nullptr;
    BinScratch bs;
    auto carve_inst_state = [&](Arena &a) {
        inst_gauss = a.take<uint32_t>((size_t)(inst_cap > 0 ? inst_cap : 1));
        inst_quad = a.take<uint8_t>((size_t)(inst_cap > 0 ? inst_cap : 1));
        ranges = a.take<uint2>(ntiles);
        tile_work = a.take<uint32_t>(ntiles);
    };
    auto carve_inst_scratch = [&](Arena &a) {
        bs.carve(a, super_cap, G.n_super);
        order = a.take<uint32_t>(ntiles);
    };
    if (counted) {
        inst_cap = (uint64_t)cap->instances;
        super_cap = cap->entries > 0 ? (uint64_t)cap->entries : inst_cap;
    }
    {
        Arena sa, ta;
        auto carve_state = [&](Arena &a) {
            gst.carve(a, n);
            if (counted) carve_inst_state(a);
        };
        auto carve_scratch = [&](Arena &a) {
            gs.carve(a, n);
            if (counted) carve_inst_scratch(a);
        };
        carve_state(sa);
        carve_scratch(ta);
        if ((rc = alloc_arena(alloc, sa.off, OMNIGS_MEM_STATE, sa, "forward state")) != OMNIGS_OK) return rc;
        carve_state(sa);
        if ((rc = alloc_arena(alloc, ta.off, OMNIGS_MEM_SCRATCH, ta, "forward scratch")) != OMNIGS_OK) return rc;
        carve_scratch(ta);
    }
    {
        // every counter and lookback word the call starts from, in one launch
        ClearList L{};
        geom_clear(n, gst, gs, L);
        if (counted) {
            bin_clear(super_cap, G, bs, L);
            L.add(cap->overflow, 1);
        }
        HIP_TRY(launch_clear(L, st));
    }
    {
        StageTimer t(st, kStProject);
        HIP_TRY(launch_project(pa, gst.rec, gs.depth_key, gst.depth, gst.n_tiles, gst.rect, gs.n_super, gst.radii,
                               gst.totals + 1, st, true));
    }
    // with capacities the binning scratch exists already: the scan of the
    // block-entry counts also partitions the emission
    ScanPartition part;
    if (counted) part = ScanPartition{bs.part, emit_blocks(super_cap)};
    if ((rc = sort_and_count(n, gst, gs, st, true, part)) != OMNIGS_OK) return rc;

    int64_t S = -1, M = -1;
    if (!counted) {
        // super entries S and tile instances M: the one host synchronisation
        uint32_t tot[3] = {0, 0, 0};
        HIP_TRY(hipMemcpyAsync(tot, gst.totals, sizeof(tot), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (tot[2]) return fail(OMNIGS_ERR_HIP, "a lookback wait of the depth sort or scan gave up (fault bits %u)", tot[2]);
        S = tot[0];
        M = tot[1];
        super_cap = (uint64_t)S;
        inst_cap = (uint64_t)M;
        Arena ia, ja;
        carve_inst_state(ia);
        carve_inst_scratch(ja);
        if ((rc = alloc_arena(alloc, ia.off, OMNIGS_MEM_STATE, ia, "instance lists")) != OMNIGS_OK) return rc;
        carve_inst_state(ia);
        if ((rc = alloc_arena(alloc, ja.off, OMNIGS_MEM_SCRATCH, ja, "binning scratch")) != OMNIGS_OK) return rc;
        carve_inst_scratch(ja);
        ClearList L{};
        bin_clear(super_cap, G, bs, L);
        HIP_TRY(launch_clear(L, st));
    }

    // the launch order (longest list first) comes out of the binning's last
    // kernel when the forward uses one
    if (!forward_uses_order(inst_cap, ntiles)) order = nullptr;
    if ((rc = run_binning(n, gst, gs, G, super_cap, inst_cap, counted, bs, ranges, inst_gauss,
                          counted ? cap->overflow : nullptr, st, true, order, ntiles, counted)) != OMNIGS_OK)
        return rc;
    {
        StageTimer t(st, kStBlendFwd);
        FrameGeom f{cam->width, pa.rows, pa.tiles_x, pa.tiles_y, 0u, pa.model == OMNIGS_CAMERA_ERP};
        HIP_TRY(launch_blend_forward(f, gst.rec, gst.depth, inst_gauss, ranges, make_blend_settings(s), out->image,
                                     out->final_T, out->n_contrib, out->n_blended, out->depth, order, tile_work,
                                     inst_cap, st, inst_quad));
    }
    state->n = n;
    state->n_instances = M;
    state->n_entries = S;
    state->width = cam->width;
    state->height = pa.rows;
    state->tiles_x = pa.tiles_x;
    state->tiles_y = pa.tiles_y;
    state->records = gst.rec;
    state->n_tiles = gst.n_tiles;
    state->depth_order = gst.order;
    state->inst_gauss = inst_gauss;
    state->inst_quad = inst_quad;
    state->tile_range = reinterpret_cast<const uint32_t *>(ranges);
    state->tile_work = tile_work;
    state->radii = gst.radii;
    state->depth = gst.depth;
    state->counts = gst.totals;
    return OMNIGS_OK;
}

omnigs_status omnigs_backward(const omnigs_gaussians *g, const omnigs_camera *cam, const omnigs_settings *s,
                              const omnigs_state *state, const omnigs_image_out *fwd, const float *dL_dimage,
                              const float *dL_ddepth, const float *dL_dalpha, omnigs_grads *grads,
                              omnigs_allocator alloc, void *stream) {
    if (!alloc.alloc) return fail(OMNIGS_ERR_INVALID, "allocator callback is NULL");
    auto carve = [&](size_t acc_words, size_t ntiles, float *&acc, uint32_t *&order) -> omnigs_status {
        Arena a;
        a.take<float>(acc_words);
        a.take<uint32_t>(ntiles);
        omnigs_status rc;
        if ((rc = alloc_arena(alloc, a.off, OMNIGS_MEM_SCRATCH, a, "gradient accumulators")) != OMNIGS_OK) return rc;
        acc = a.take<float>(acc_words);
        order = a.take<uint32_t>(ntiles);
        return OMNIGS_OK;
    };
    return backward_impl(g, cam, s, state, fwd, dL_dimage, dL_ddepth, dL_dalpha, grads, stream, carve);
}

omnigs_status omnigs_backward_noalloc(const omnigs_gaussians *g, const omnigs_camera *cam,
                                      const omnigs_settings *s, const omnigs_state *state,
                                      const omnigs_image_out *fwd, const float *dL_dimage, const float *dL_ddepth,
                                      const float *dL_dalpha, omnigs_grads *grads, void *stream) {
    auto carve = [&](size_t acc_words, size_t ntiles, float *&acc, uint32_t *&order) -> omnigs_status {
        Arena a;
        a.take<float>(acc_words);
        a.take<uint32_t>(ntiles);
        if (a.off > kNoAllocScratchBytes)
            return fail(OMNIGS_ERR_INVALID,
                        "omnigs_backward_noalloc: %zu Gaussians and %zu tiles need %zu bytes of accumulators and "
                        "tile order, more than its %zu-byte device scratch",
                        (size_t)g->n, ntiles, a.off, kNoAllocScratchBytes);
        char *base = nullptr;
        omnigs_status rc;
        if ((rc = noalloc_scratch(base)) != OMNIGS_OK) return rc;
        a.base = base;
        a.off = 0;
        acc = a.take<float>(acc_words);
        order = a.take<uint32_t>(ntiles);
        return OMNIGS_OK;
    };
    return backward_impl(g, cam, s, state, fwd, dL_dimage, dL_ddepth, dL_dalpha, grads, stream, carve);
}

omnigs_status omnigs_l1_loss(const float *image, const float *target, int64_t count, float *dL_dimage, float *loss,
                             omnigs_allocator alloc, void *stream) {
    if (!image || !target || !loss) return fail(OMNIGS_ERR_INVALID, "image, target or loss is NULL");
    if (count <= 0) return fail(OMNIGS_ERR_INVALID, "count must be positive");
    if (!alloc.alloc) return fail(OMNIGS_ERR_INVALID, "allocator callback is NULL");
    Arena a;
    omnigs_status rc;
    if ((rc = alloc_arena(alloc, l1_scratch_bytes(), OMNIGS_MEM_SCRATCH, a, "loss partial sums")) != OMNIGS_OK)
        return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StageTimer t(st, kStL1);
    HIP_TRY(launch_l1(image, target, count, dL_dimage, loss, a.base, st));
    return OMNIGS_OK;
}

omnigs_status omnigs_set_cover_key_blocks(uint32_t blocks) {
    g_cover_key_blocks = blocks == 0 || blocks > kMaxCoverKeyBlocks ? kMaxCoverKeyBlocks : blocks;
    return OMNIGS_OK;
}

omnigs_status omnigs_selftest_lookback(int32_t primitive, int64_t n, uint32_t max_polls, omnigs_allocator alloc,
                                       uint32_t *fault, int32_t *correct, void *stream) {
    if (primitive != 0 && primitive != 1) return fail(OMNIGS_ERR_INVALID, "primitive must be 0 (sort) or 1 (scan)");
    if (n < 1 || n > (int64_t(1) << 26)) return fail(OMNIGS_ERR_INVALID, "n = %lld not in [1, 2^26]", (long long)n);
    if (!fault || !correct) return fail(OMNIGS_ERR_INVALID, "fault or correct is NULL");
    if (!alloc.alloc) return fail(OMNIGS_ERR_INVALID, "allocator callback is NULL");
    static std::mutex selftest_mutex;
    std::lock_guard<std::mutex> lock(selftest_mutex);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t m = (size_t)n;
    Arena a;
    uint32_t *keys, *vals, *kt, *vt, *ko, *vo, *word;
    void *tmp;
    auto carve = [&](Arena &ar) {
        keys = ar.take<uint32_t>(m);
        vals = ar.take<uint32_t>(m + 1);
        kt = ar.take<uint32_t>(m);
        vt = ar.take<uint32_t>(m);
        ko = ar.take<uint32_t>(m);
        vo = ar.take<uint32_t>(m);
        word = ar.take<uint32_t>(1);
        tmp = ar.take_bytes(std::max(sort_scratch_bytes(n), scan_scratch_bytes(n)));
    };
    carve(a);
    omnigs_status rc;
    if ((rc = alloc_arena(alloc, a.off, OMNIGS_MEM_SCRATCH, a, "self-test buffers")) != OMNIGS_OK) return rc;
    carve(a);
    const uint32_t mask = primitive == 0 ? 0xffffffffu : 15u;
    HIP_TRY(launch_selftest_keys(keys, n, mask, st));
    HIP_TRY(launch_fill_u32(word, 0u, 1, st));
    set_lookback_poll_limit(max_polls);
    hipError_t e = primitive == 0 ? radix_sort_pairs(keys, nullptr, kt, vt, ko, vo, n, 32, tmp, st, nullptr, nullptr, 0,
                                                     false, word)
                                  : scan_exclusive(keys, vals, n, vals + n, tmp, st, nullptr, false, word);
    set_lookback_poll_limit(0);
    HIP_TRY(e);
    std::vector<uint32_t> hk(primitive == 0 ? m : 0), hv(primitive == 0 ? m : m + 1);
    if (primitive == 0) {
        HIP_TRY(hipMemcpyAsync(hk.data(), ko, m * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hv.data(), vo, m * 4, hipMemcpyDeviceToHost, st));
    } else {
        HIP_TRY(hipMemcpyAsync(hv.data(), vals, (m + 1) * 4, hipMemcpyDeviceToHost, st));
    }
    HIP_TRY(hipMemcpyAsync(fault, word, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    bool ok = true;
    if (primitive == 0) {
        // ascending keys, a stable permutation of the input
        std::vector<char> seen(m, 0);
        for (size_t i = 0; i < m && ok; ++i) {
            const uint32_t v = hv[i];
            ok = v < m && !seen[v] && hk[i] == selftest_key(v);
            if (ok) seen[v] = 1;
            if (ok && i > 0) ok = hk[i - 1] < hk[i] || (hk[i - 1] == hk[i] && hv[i - 1] < v);
        }
    } else {
        uint64_t run = 0;
        for (size_t i = 0; i <= m && ok; ++i) {
            ok = hv[i] == (uint32_t)run;
            if (i < m) run += selftest_key((uint32_t)i) & mask;
        }
    }
    *correct = ok ? 1 : 0;
    return OMNIGS_OK;
}

omnigs_status omnigs_measure_ceilings(int64_t atomic_words, int64_t copy_bytes, int32_t repeats,
                                      omnigs_allocator alloc, omnigs_ceilings *out, void *stream) {
    if (!out) return fail(OMNIGS_ERR_INVALID, "out is NULL");
    if (repeats < 1) return fail(OMNIGS_ERR_INVALID, "repeats must be >= 1");
    if (atomic_words < 0 || atomic_words >= (int64_t(1) << 32))
        return fail(OMNIGS_ERR_INVALID, "atomic_words %lld out of range", (long long)atomic_words);
    if (copy_bytes < 0 || copy_bytes % 16 != 0)
        return fail(OMNIGS_ERR_INVALID, "copy_bytes must be a non-negative multiple of 16");
    if (!alloc.alloc) return fail(OMNIGS_ERR_INVALID, "allocator callback is NULL");
    Arena a;
    auto carve = [&](Arena &ar, float *&abuf, float *&src, float *&dst) {
        abuf = atomic_words ? ar.take<float>((size_t)atomic_words) : nullptr;
        src = copy_bytes ? ar.take<float>((size_t)copy_bytes / 4) : nullptr;
        dst = copy_bytes ? ar.take<float>((size_t)copy_bytes / 4) : nullptr;
    };
    float *abuf, *src, *dst;
    carve(a, abuf, src, dst);
    omnigs_status rc;
    if ((rc = alloc_arena(alloc, a.off, OMNIGS_MEM_SCRATCH, a, "ceiling buffers")) != OMNIGS_OK) return rc;
    carve(a, abuf, src, dst);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (abuf) HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(abuf), 0u, atomic_words, st));
    if (src) HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(src), 0u, copy_bytes / 4, st));
    double ms[4], work[4];
    HIP_TRY(measure_ceilings(abuf, (uint32_t)atomic_words, src, dst, copy_bytes, repeats, ms, work, st));
    auto rate = [&](int k) { return ms[k] > 0.0 ? work[k] / (ms[k] * 1e-3) : 0.0; };
    out->fma_tflops = rate(0) / 1e12;
    out->exp_gops = rate(1) / 1e9;
    out->atomic_gops = rate(2) / 1e9;
    out->copy_gbps = rate(3) / 1e9;
    return OMNIGS_OK;
}

omnigs_status omnigs_photometric_loss(const float *image, const float *target, int32_t channels, int32_t height,
                                      int32_t width, double lambda, const float *mask, float *dL_dimage, float *loss,
                                      omnigs_allocator alloc, void *stream) {
    if (!image || !target || !loss) return fail(OMNIGS_ERR_INVALID, "image, target or loss is NULL");
    if (channels < 1 || height < 1 || width < 1 || channels > 64 || height > 65520 || width > 65520)
        return fail(OMNIGS_ERR_INVALID, "image size out of range");
    if (!(lambda >= 0.0 && lambda <= 1.0)) return fail(OMNIGS_ERR_INVALID, "lambda must be in [0, 1]");
    if (!alloc.alloc) return fail(OMNIGS_ERR_INVALID, "allocator callback is NULL");
    Arena a;
    omnigs_status rc;
    if ((rc = alloc_arena(alloc, ssim_scratch_bytes(channels, height, width, dL_dimage != nullptr), OMNIGS_MEM_SCRATCH,
                          a, "loss planes and partial sums")) != OMNIGS_OK)
        return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StageTimer t(st, kStL1);
    HIP_TRY(launch_photometric(image, target, mask, channels, height, width, (float)lambda, dL_dimage, loss, a.base,
                               st));
    return OMNIGS_OK;
}

omnigs_status omnigs_forward_batch_bytes(int64_t n, const omnigs_camera *cams, int32_t batch,
                                         int64_t instance_capacity, uint64_t *bytes) {
    if (!bytes) return fail(OMNIGS_ERR_INVALID, "bytes is NULL");
    *bytes = 0;
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(OMNIGS_ERR_INVALID, "n = %lld out of range", (long long)n);
    if (instance_capacity < 1 || instance_capacity >= (int64_t(1) << 32))
        return fail(OMNIGS_ERR_INVALID, "instance_capacity %lld not in [1, 2^32)", (long long)instance_capacity);
    Grids G;
    uint64_t total_tiles = 0;
    omnigs_status rc;
    if ((rc = batch_grids(cams, batch, n, G, total_tiles)) != OMNIGS_OK) return rc;
    const int64_t nrec = n * batch;
    if (nrec >= (int64_t(1) << 32) - 1) return fail(OMNIGS_ERR_INVALID, "batch * n must stay below 2^32");
    BatchBuffers bb;
    Arena ra, ia;
    bb.carve_records(ra, nrec);
    bb.carve_instances(ia, (uint64_t)instance_capacity, (uint64_t)instance_capacity, (uint32_t)total_tiles, G);
    *bytes = arena_request(ra.off) + arena_request(ia.off);
    return OMNIGS_OK;
}

omnigs_status omnigs_forward_batch(const omnigs_gaussians *g, const omnigs_camera *cams, int32_t batch,
                                   const omnigs_settings *s, omnigs_allocator alloc, omnigs_image_out *outs,
                                   int64_t instance_capacity, int32_t *overflow, int64_t *n_instances,
                                   void *stream) {
    omnigs_status rc;
    if (n_instances) *n_instances = -1;
    if ((rc = check_gaussians(g)) != OMNIGS_OK) return rc;
    if ((rc = check_settings(s)) != OMNIGS_OK) return rc;
    if (!cams || !outs) return fail(OMNIGS_ERR_INVALID, "cameras or outputs is NULL");
    if (!alloc.alloc) return fail(OMNIGS_ERR_INVALID, "allocator callback is NULL");
    if (instance_capacity < 0 || instance_capacity >= (int64_t(1) << 32))
        return fail(OMNIGS_ERR_INVALID, "instance_capacity %lld out of range", (long long)instance_capacity);
    const int64_t n = g->n;
    Grids G;
    uint64_t total_tiles = 0;
    if ((rc = batch_grids(cams, batch, n, G, total_tiles)) != OMNIGS_OK) return rc;
    const int64_t nrec = n * batch;  // record b * n + i: camera b, Gaussian i
    if (nrec >= (int64_t(1) << 32) - 1) return fail(OMNIGS_ERR_INVALID, "batch * n must stay below 2^32");
    FrameGeom frames[kMaxBatch];
    CamTable ct{};
    ct.count = batch;
    for (int b = 0; b < batch; ++b) {
        if (!outs[b].image || !outs[b].final_T || !outs[b].n_contrib)
            return fail(OMNIGS_ERR_INVALID, "output pointer of camera %d is NULL", b);
        if ((outs[b].depth != nullptr) != (outs[0].depth != nullptr))
            return fail(OMNIGS_ERR_INVALID, "depth images must be requested for every camera of a batch or for none");
        const ProjectArgs pb = make_project_args(g, &cams[b], s);
        CamGeom &cg = ct.c[b];
        for (int k = 0; k < 9; ++k) cg.R[k] = pb.R[k];
        for (int k = 0; k < 3; ++k) {
            cg.t[k] = pb.t[k];
            cg.campos[k] = pb.campos[k];
        }
        cg.width = pb.width;
        cg.height = pb.height;
        cg.rows = pb.rows;
        cg.tiles_x = pb.tiles_x;
        cg.tiles_y = pb.tiles_y;
        cg.model = pb.model;
        cg.fx = pb.fx;
        cg.fy = pb.fy;
        cg.cx = pb.cx;
        cg.cy = pb.cy;
        frames[b] = FrameGeom{pb.width, pb.rows, pb.tiles_x, pb.tiles_y, G.sup.f[b].tile_base,
                              pb.model == OMNIGS_CAMERA_ERP};
    }
    const ProjectArgs pa = make_project_args(g, &cams[0], s);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t ntiles = (uint32_t)total_tiles;

    // per-record buffers (all scratch: no backward state is kept)
    BatchBuffers bb;
    GeomState &gst = bb.gst;
    GeomScratch &gs = bb.gs;
    Arena ra;
    bb.carve_records(ra, nrec);
    if ((rc = alloc_arena(alloc, ra.off, OMNIGS_MEM_SCRATCH, ra, "per-record scratch")) != OMNIGS_OK) return rc;
    bb.carve_records(ra, nrec);
    if (overflow) HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(overflow), 0u, 1, st));
    HIP_TRY(launch_fill_u32(gst.totals + 2, 0u, 1, st));  // fault bits
    {
        StageTimer t(st, kStProject);
        HIP_TRY(launch_project_batch(pa, ct, gst.rec, gs.depth_key, gst.depth, gst.n_tiles, gst.rect, gs.n_super,
                                     gst.totals + 1,
                                     st));
    }
    if ((rc = sort_and_count(nrec, gst, gs, st)) != OMNIGS_OK) return rc;
    // capacities: read back (exact), or the caller's instance capacity for
    // both levels, counted on the device: every block entry holds at least
    // one covered tile (a rectangle that wraps across the seam reaches the
    // last tile column and misses fewer than 8 columns), so S <= M
    uint64_t super_cap, inst_cap;
    const bool counted = instance_capacity > 0;
    if (!counted) {
        uint32_t tot[3] = {0, 0, 0};
        HIP_TRY(hipMemcpyAsync(tot, gst.totals, sizeof(tot), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (tot[2]) return fail(OMNIGS_ERR_HIP, "a lookback wait of the depth sort or scan gave up (fault bits %u)", tot[2]);
        super_cap = tot[0];
        inst_cap = tot[1];
        if (n_instances) *n_instances = tot[1];
    } else {
        inst_cap = (uint64_t)instance_capacity;
        super_cap = inst_cap;
    }
    Arena ia;
    bb.carve_instances(ia, inst_cap, super_cap, ntiles, G);
    if ((rc = alloc_arena(alloc, ia.off, OMNIGS_MEM_SCRATCH, ia, "instance lists")) != OMNIGS_OK) return rc;
    bb.carve_instances(ia, inst_cap, super_cap, ntiles, G);
    if ((rc = run_binning(nrec, gst, gs, G, super_cap, inst_cap, counted, bb.bs, bb.ranges, bb.inst_gauss, overflow,
                          st, false, bb.order, ntiles)) != OMNIGS_OK)
        return rc;
    {
        StageTimer t(st, kStBlendFwd);
        HIP_TRY(launch_blend_forward_frames(frames, outs, batch, gst.rec, gst.depth, bb.inst_gauss, bb.ranges,
                                            make_blend_settings(s), bb.order, ntiles, st));
    }
    return OMNIGS_OK;
}

// ---------------------------------------------------------- optimisation
}  // extern "C"

namespace {

omnigs_status check_params(const omnigs_params *p, const char *what) {
    if (!p) return fail(OMNIGS_ERR_INVALID, "%s is NULL", what);
    if (p->n < 0 || p->n >= (int64_t(1) << 31)) return fail(OMNIGS_ERR_INVALID, "%s: n out of range", what);
    if (p->sh_coeffs < 1 || p->sh_coeffs > 16) return fail(OMNIGS_ERR_INVALID, "%s: sh_coeffs out of range", what);
    if (p->n > 0 && (!p->means || !p->log_scales || !p->quats || !p->logits || !p->sh))
        return fail(OMNIGS_ERR_INVALID, "%s: a parameter pointer is NULL", what);
    return OMNIGS_OK;
}

OptimArrays arrays_of(const omnigs_params *p) {
    return OptimArrays{{p->means, p->log_scales, p->quats, p->logits, p->sh}};
}

omnigs_status same_shape(const omnigs_params *a, const omnigs_params *b, const char *what) {
    if (a->n != b->n || a->sh_coeffs != b->sh_coeffs) return fail(OMNIGS_ERR_INVALID, "%s: shape mismatch", what);
    return OMNIGS_OK;
}

}  // namespace

extern "C" {

omnigs_status omnigs_adam_step(omnigs_params *p, const omnigs_grads *g, omnigs_params *m1, omnigs_params *m2,
                               const omnigs_adam_settings *s, omnigs_gaussians *act, const int32_t *skip,
                               void *stream) {
    omnigs_status rc;
    if ((rc = check_params(p, "params")) != OMNIGS_OK || (rc = check_params(m1, "m1")) != OMNIGS_OK ||
        (rc = check_params(m2, "m2")) != OMNIGS_OK)
        return rc;
    if ((rc = same_shape(p, m1, "m1")) != OMNIGS_OK || (rc = same_shape(p, m2, "m2")) != OMNIGS_OK) return rc;
    if (!g || !s) return fail(OMNIGS_ERR_INVALID, "gradients or settings is NULL");
    if (p->n > 0 && (!g->dmeans || !g->dscales || !g->dquats || !g->dopacities || !g->dsh))
        return fail(OMNIGS_ERR_INVALID, "a gradient pointer is NULL");
    if (s->step < 1) return fail(OMNIGS_ERR_INVALID, "step must be >= 1");
    if (!(s->beta1 >= 0.0 && s->beta1 < 1.0 && s->beta2 >= 0.0 && s->beta2 < 1.0 && s->eps >= 0.0))
        return fail(OMNIGS_ERR_INVALID, "bad Adam coefficients");
    const int64_t n = p->n;
    const int64_t shf = (int64_t)p->sh_coeffs * 3;
    AdamArgs a{};
    const int64_t len[kSegments] = {3 * n, 3 * n, 4 * n, n, shf * n};
    int64_t off = 0;
    for (int k = 0; k < kSegments; ++k) {
        a.begin[k] = off;
        off += len[k];
    }
    a.total = off;
    a.lr[kSegMeans] = (float)s->lr_means;
    a.lr[kSegLogScales] = (float)s->lr_log_scales;
    a.lr[kSegQuats] = (float)s->lr_quats;
    a.lr[kSegLogits] = (float)s->lr_logits;
    a.lr[kSegSh] = (float)s->lr_sh_dc;
    a.lr_sh_rest = (float)s->lr_sh_rest;
    a.sh_stride = shf;
    a.beta1 = (float)s->beta1;
    a.beta2 = (float)s->beta2;
    a.eps = (float)s->eps;
    a.inv_bc1 = (float)(1.0 / (1.0 - std::pow(s->beta1, s->step)));
    a.inv_sqrt_bc2 = (float)(1.0 / std::sqrt(1.0 - std::pow(s->beta2, s->step)));
    const OptimArrays G{{g->dmeans, g->dscales, g->dquats, g->dopacities, g->dsh}};
    StageTimer t(static_cast<hipStream_t>(stream), kStAdam);
    HIP_TRY(launch_adam(arrays_of(p), G, arrays_of(m1), arrays_of(m2), a,
                        act ? const_cast<float *>(act->scales) : nullptr,
                        act ? const_cast<float *>(act->opacities) : nullptr, skip, static_cast<hipStream_t>(stream)));
    return OMNIGS_OK;
}

omnigs_status omnigs_accumulate_stats(const omnigs_state *state, const omnigs_grads *g,
                                      omnigs_densify_stats *stats, const int32_t *skip, void *stream) {
    if (!state || !g || !stats) return fail(OMNIGS_ERR_INVALID, "state, gradients or statistics is NULL");
    if (state->n > 0 && (!state->n_tiles || !state->radii || !g->dscreen || !stats->accum || !stats->denom ||
                         !stats->max_radius))
        return fail(OMNIGS_ERR_INVALID, "a state, gradient or statistics pointer is NULL");
    StageTimer t(static_cast<hipStream_t>(stream), kStStats);
    HIP_TRY(launch_stats(state->n_tiles, state->radii, g->dscreen, state->n, stats->accum, stats->denom,
                         stats->max_radius, skip, static_cast<hipStream_t>(stream)));
    return OMNIGS_OK;
}

omnigs_status omnigs_densify(const omnigs_params *p, const omnigs_params *m1, const omnigs_params *m2,
                             const omnigs_densify_stats *stats, const float *noise, const omnigs_densify_settings *s,
                             omnigs_allocator alloc, omnigs_params *p_out, omnigs_params *m1_out,
                             omnigs_params *m2_out, omnigs_densify_stats *stats_out, int64_t *n_out, void *stream) {
    omnigs_status rc;
    if ((rc = check_params(p, "params")) != OMNIGS_OK || (rc = check_params(m1, "m1")) != OMNIGS_OK ||
        (rc = check_params(m2, "m2")) != OMNIGS_OK)
        return rc;
    if ((rc = same_shape(p, m1, "m1")) != OMNIGS_OK || (rc = same_shape(p, m2, "m2")) != OMNIGS_OK) return rc;
    if (!stats || !s || !p_out || !m1_out || !m2_out || !stats_out || !n_out || !alloc.alloc)
        return fail(OMNIGS_ERR_INVALID, "a statistics, settings, output or allocator argument is NULL");
    const int64_t n = p->n;
    if (n > 0 && (!noise || !stats->accum || !stats->denom || !stats->max_radius))
        return fail(OMNIGS_ERR_INVALID, "noise or a statistics array is NULL");
    if (!(s->grad_threshold >= 0.0 && s->percent_dense > 0.0 && s->extent > 0.0 && s->min_opacity > 0.0 &&
          s->min_opacity < 1.0 && s->big_fraction > 0.0 && s->split_shrink > 0.0))
        return fail(OMNIGS_ERR_INVALID, "bad densification settings");
    if ((int64_t)4 * n >= (int64_t(1) << 32)) return fail(OMNIGS_ERR_INVALID, "too many Gaussians");
    hipStream_t st = static_cast<hipStream_t>(stream);
    StageTimer timer(st, kStDensify);
    const int shf = p->sh_coeffs * 3;
    // thresholds rounded once to float32: the decisions compare float32
    // values (log-scales, logits, radii, the averaged gradient)
    DensifyArgs d{};
    d.tau = (float)s->grad_threshold;
    d.log_clone = (float)std::log(s->percent_dense * s->extent);
    d.logit_min = (float)std::log(s->min_opacity / (1.0 - s->min_opacity));
    d.screen_on = s->max_screen > 0.0;
    d.max_screen = (float)s->max_screen;
    d.log_big = (float)std::log(s->big_fraction * s->extent);
    d.log_shrink = (float)std::log(s->split_shrink);
    Arena a;
    a.take<uint32_t>((size_t)(4 * n + 1));
    a.take<uint32_t>((size_t)(4 * n + 2));
    a.take_bytes(scan_scratch_bytes(4 * n + 1));
    if ((rc = alloc_arena(alloc, a.off, OMNIGS_MEM_SCRATCH, a, "densification scratch")) != OMNIGS_OK) return rc;
    uint32_t *flags = a.take<uint32_t>((size_t)(4 * n + 1));
    uint32_t *pos = a.take<uint32_t>((size_t)(4 * n + 2));  // scan, total, fault bits
    void *scan_tmp = a.take_bytes(scan_scratch_bytes(4 * n + 1));
    const OptimArrays P = arrays_of(p);
    HIP_TRY(launch_dens_flags(P, stats->accum, stats->denom, stats->max_radius, n, d, flags, st));
    HIP_TRY(launch_fill_u32(pos + 4 * n + 1, 0u, 1, st));
    HIP_TRY(scan_exclusive(flags, pos, 4 * n, pos + 4 * n, scan_tmp, st, nullptr, false, pos + 4 * n + 1));
    uint32_t tot[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(tot, pos + 4 * n, sizeof(tot), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (tot[1]) return fail(OMNIGS_ERR_HIP, "a lookback wait of the densification scan gave up");
    const int64_t no = tot[0];
    // outputs: parameters, two moment sets, statistics
    Arena o;
    auto carve = [&](Arena &ar, omnigs_params *q) {
        q->means = ar.take<float>((size_t)(3 * (no > 0 ? no : 1)));
        q->log_scales = ar.take<float>((size_t)(3 * (no > 0 ? no : 1)));
        q->quats = ar.take<float>((size_t)(4 * (no > 0 ? no : 1)));
        q->logits = ar.take<float>((size_t)(no > 0 ? no : 1));
        q->sh = ar.take<float>((size_t)shf * (no > 0 ? no : 1));
        q->n = no;
        q->sh_degree = p->sh_degree;
        q->sh_coeffs = p->sh_coeffs;
    };
    auto carve_all = [&](Arena &ar) {
        carve(ar, p_out);
        carve(ar, m1_out);
        carve(ar, m2_out);
        stats_out->accum = ar.take<float>((size_t)(no > 0 ? no : 1));
        stats_out->denom = ar.take<float>((size_t)(no > 0 ? no : 1));
        stats_out->max_radius = ar.take<float>((size_t)(no > 0 ? no : 1));
    };
    carve_all(o);
    if ((rc = alloc_arena(alloc, o.off, OMNIGS_MEM_STATE, o, "densified parameters")) != OMNIGS_OK) return rc;
    carve_all(o);
    HIP_TRY(launch_dens_scatter(P, arrays_of(m1), arrays_of(m2), flags, pos, noise, n, shf, d.log_shrink,
                                arrays_of(p_out), arrays_of(m1_out), arrays_of(m2_out), st));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(stats_out->accum), 0u, no, st));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(stats_out->denom), 0u, no, st));
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(stats_out->max_radius), 0u, no, st));
    *n_out = no;
    return OMNIGS_OK;
}

omnigs_status omnigs_reset_opacity(omnigs_params *p, omnigs_params *m1, omnigs_params *m2, double value,
                                   void *stream) {
    omnigs_status rc;
    if ((rc = check_params(p, "params")) != OMNIGS_OK || (rc = check_params(m1, "m1")) != OMNIGS_OK ||
        (rc = check_params(m2, "m2")) != OMNIGS_OK)
        return rc;
    if ((rc = same_shape(p, m1, "m1")) != OMNIGS_OK || (rc = same_shape(p, m2, "m2")) != OMNIGS_OK) return rc;
    if (!(value > 0.0 && value < 1.0)) return fail(OMNIGS_ERR_INVALID, "reset value must be in (0, 1)");
    HIP_TRY(launch_reset_opacity(p->logits, m1->logits, m2->logits, p->n, (float)std::log(value / (1.0 - value)),
                                 static_cast<hipStream_t>(stream)));
    return OMNIGS_OK;
}

omnigs_status omnigs_profile_enable(uint32_t stages) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.stages.store(stages, std::memory_order_relaxed);
    return OMNIGS_OK;
}

int32_t omnigs_profile_num_stages(void) { return kStCount; }

const char *omnigs_profile_stage_name(int32_t stage) {
    if (stage < 0 || stage >= kStCount) return "";
    return kStageNames[stage];
}

omnigs_status omnigs_profile_read(double *ms, int64_t *launches) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    for (auto &r : g_prof.pending) {
        HIP_TRY(hipEventSynchronize(r.b));
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
        g_prof.ms[r.stage] += t;
        g_prof.launches[r.stage] += 1;
        g_prof.pool.push_back(r.a);
        g_prof.pool.push_back(r.b);
    }
    g_prof.pending.clear();
    for (int k = 0; k < kStCount; ++k) {
        if (ms) ms[k] = g_prof.ms[k];
        if (launches) launches[k] = g_prof.launches[k];
        g_prof.ms[k] = 0.0;
        g_prof.launches[k] = 0;
    }
    return OMNIGS_OK;
}

}  // extern "C"
