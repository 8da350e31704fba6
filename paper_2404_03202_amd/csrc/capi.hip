// capi.hip -- the extern "C" entry points of libomnigs.so (include/omnigs.h):
// argument validation, carving of caller-allocated device memory, stage
// sequencing on the caller's stream, optional per-stage HIP-event timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
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
    kStEmit,
    kStTileSort,
    kStRanges,
    kStTileOrder,
    kStBlendFwd,
    kStL1,
    kStBwdClear,
    kStBlendBwd,
    kStProjectBwd,
    kStCount
};
const char *kStageNames[kStCount] = {"project",    "depth_sort", "emit_count", "emit",      "tile_sort",
                                     "tile_ranges", "tile_order", "blend_fwd",  "l1_loss",   "bwd_clear",
                                     "blend_bwd",  "project_bwd"};

struct Profiler {
    std::mutex mu;
    bool on = false;
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
        if (!g_prof.on) return;
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
    if (c->width <= 0 || c->width % kTile != 0 || c->width > 65520)
        return fail(OMNIGS_ERR_INVALID, "width %d must be a positive multiple of 16, <= 65520", c->width);
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
    if (!(s->T_min > 0.0 && s->T_min < 1.0)) return fail(OMNIGS_ERR_INVALID, "T_min must be in (0, 1)");
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
    a.tiles_x = c->width / kTile;
    a.tiles_y = (c->height + kTile - 1) / kTile;
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

// N-sized buffers of one forward: persistent part (state) and scratch.
struct GeomState {
    BlendRecord *rec;
    uint32_t *n_tiles, *order;
    uint2 *rect;
    void carve(Arena &a, int64_t n) {
        const size_t m = (size_t)(n > 0 ? n : 1);
        rec = a.take<BlendRecord>(m);
        n_tiles = a.take<uint32_t>(m);
        order = a.take<uint32_t>(m);
        rect = a.take<uint2>(m);
    }
};
struct GeomScratch {
    uint32_t *depth_key, *iota, *keys_tmp, *vals_tmp, *keys_sorted, *offs;
    void *sort_tmp, *scan_tmp;
    void carve(Arena &a, int64_t n) {
        const size_t m = (size_t)(n > 0 ? n : 1);
        depth_key = a.take<uint32_t>(m);
        iota = a.take<uint32_t>(m);
        keys_tmp = a.take<uint32_t>(m);
        vals_tmp = a.take<uint32_t>(m);
        keys_sorted = a.take<uint32_t>(m);
        offs = a.take<uint32_t>(m + 1);
        sort_tmp = a.take_bytes(sort_scratch_bytes((int64_t)m));
        scan_tmp = a.take_bytes(scan_scratch_bytes((int64_t)m));
    }
};

// Projection, depth sort and per-rank instance offsets of one camera.
// Leaves the instance total M in gs.offs[n].
omnigs_status run_geometry(const ProjectArgs &pa, GeomState &gst, GeomScratch &gs, hipStream_t st) {
    const int64_t n = pa.n;
    {
        StageTimer t(st, kStProject);
        HIP_TRY(launch_project(pa, gst.rec, gs.depth_key, gst.n_tiles, gst.rect, st));
    }
    {
        StageTimer t(st, kStDepthSort);
        HIP_TRY(launch_iota(gs.iota, n, st));
        HIP_TRY(radix_sort_pairs(gs.depth_key, gs.iota, gs.keys_tmp, gs.vals_tmp, gs.keys_sorted, gst.order, n, 32,
                                 gs.sort_tmp, st));
    }
    {
        StageTimer t(st, kStEmitCount);
        HIP_TRY(scan_exclusive(gst.n_tiles, gs.offs, n, gs.offs + n, gs.scan_tmp, st, gst.order));
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
                             omnigs_allocator alloc, omnigs_image_out *out, omnigs_state *state, void *stream) {
    omnigs_status rc;
    if ((rc = check_gaussians(g)) != OMNIGS_OK) return rc;
    if ((rc = check_camera(cam)) != OMNIGS_OK) return rc;
    if ((rc = check_settings(s)) != OMNIGS_OK) return rc;
    if (!alloc.alloc) return fail(OMNIGS_ERR_INVALID, "allocator callback is NULL");
    if (!out || !out->image || !out->final_T || !out->n_contrib) return fail(OMNIGS_ERR_INVALID, "output pointer is NULL");
    if (!state) return fail(OMNIGS_ERR_INVALID, "state is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const ProjectArgs pa = make_project_args(g, cam, s);
    const int64_t n = g->n;
    const uint32_t ntiles = (uint32_t)(pa.tiles_x * pa.tiles_y);

    // N-sized buffers
    Arena sa, ta;
    GeomState gst;
    GeomScratch gs;
    gst.carve(sa, n);
    const size_t geom_state_bytes = sa.off;
    gs.carve(ta, n);
    const size_t geom_scratch_bytes = ta.off;
    if ((rc = alloc_arena(alloc, geom_state_bytes, OMNIGS_MEM_STATE, sa, "per-Gaussian state")) != OMNIGS_OK) return rc;
    gst.carve(sa, n);
    if ((rc = alloc_arena(alloc, geom_scratch_bytes, OMNIGS_MEM_SCRATCH, ta, "per-Gaussian scratch")) != OMNIGS_OK)
        return rc;
    gs.carve(ta, n);

    if ((rc = run_geometry(pa, gst, gs, st)) != OMNIGS_OK) return rc;

    // instance count: the one host synchronisation
    uint32_t m32 = 0;
    HIP_TRY(hipMemcpyAsync(&m32, gs.offs + n, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const int64_t M = m32;

    // M-sized buffers
    const int bits = bits_for(ntiles);
    const int passes = (bits + 7) / 8;
    Arena ia, ja;
    uint32_t *tile_work;
    auto carve_inst = [&](Arena &a, uint32_t *&tile, uint32_t *&gauss, uint2 *&ranges) {
        tile = a.take<uint32_t>((size_t)(M > 0 ? M : 1));
        gauss = a.take<uint32_t>((size_t)(M > 0 ? M : 1));
        ranges = a.take<uint2>(ntiles);
        tile_work = a.take<uint32_t>(ntiles);
    };
    uint32_t *inst_tile, *inst_gauss, *tmp_tile, *tmp_gauss;
    uint2 *ranges;
    void *sort_tmp;
    carve_inst(ia, inst_tile, inst_gauss, ranges);
    const size_t inst_state_bytes = ia.off;
    uint32_t *part, *order;
    auto carve_tmp = [&](Arena &a) {
        tmp_tile = a.take<uint32_t>((size_t)(M > 0 ? M : 1));
        tmp_gauss = a.take<uint32_t>((size_t)(M > 0 ? M : 1));
        sort_tmp = a.take_bytes(sort_scratch_bytes(M));
        part = a.take<uint32_t>((size_t)emit_blocks((uint64_t)M) + 1);
        order = a.take<uint32_t>(ntiles);
    };
    carve_tmp(ja);
    const size_t inst_scratch_bytes = ja.off;
    if ((rc = alloc_arena(alloc, inst_state_bytes, OMNIGS_MEM_STATE, ia, "instance lists")) != OMNIGS_OK) return rc;
    carve_inst(ia, inst_tile, inst_gauss, ranges);
    if ((rc = alloc_arena(alloc, inst_scratch_bytes, OMNIGS_MEM_SCRATCH, ja, "instance sort scratch")) != OMNIGS_OK)
        return rc;
    carve_tmp(ja);

    {
        StageTimer t(st, kStEmit);
        // emit where the ping-pong of the tile sort starts, so that the
        // last pass lands in the state buffers
        uint32_t *et = (passes % 2) ? tmp_tile : inst_tile;
        uint32_t *eg = (passes % 2) ? tmp_gauss : inst_gauss;
        EmitFrames ef{};
        ef.n_per = n > 0 ? n : 1;
        ef.count = 1;
        ef.tiles_x[0] = pa.tiles_x;
        ef.tile_base[0] = 0u;
        HIP_TRY(launch_emit(gst.order, gst.n_tiles, gst.rect, gs.offs, n, part, gs.offs + n, ef, (uint64_t)M, et, eg,
                            nullptr, st));
    }
    {
        StageTimer t(st, kStTileSort);
        // odd pass counts start from the scratch pair, even ones from the
        // state pair; the ping-pong never reads and writes one buffer
        const bool odd = passes % 2;
        HIP_TRY(radix_sort_pairs(odd ? tmp_tile : inst_tile, odd ? tmp_gauss : inst_gauss, tmp_tile, tmp_gauss,
                                 inst_tile, inst_gauss, M, bits, sort_tmp, st));
    }
    {
        StageTimer t(st, kStRanges);
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(ranges), 0u, 2 * (int64_t)ntiles, st));
        HIP_TRY(launch_tile_ranges(inst_tile, gs.offs + n, (uint64_t)M, ranges, ntiles, st));
    }
    {
        StageTimer t(st, kStTileOrder);
        HIP_TRY(launch_tile_order(ranges, nullptr, ntiles, order, st));
    }
    {
        StageTimer t(st, kStBlendFwd);
        FrameGeom f{cam->width, cam->height, pa.tiles_x, pa.tiles_y, 0u};
        HIP_TRY(launch_blend_forward(f, gst.rec, inst_gauss, ranges, make_blend_settings(s), out->image, out->final_T,
                                     out->n_contrib, out->n_blended, order, tile_work, st));
    }
    state->n = n;
    state->n_instances = M;
    state->width = cam->width;
    state->height = cam->height;
    state->tiles_x = pa.tiles_x;
    state->tiles_y = pa.tiles_y;
    state->records = gst.rec;
    state->n_tiles = gst.n_tiles;
    state->depth_order = gst.order;
    state->inst_tile = inst_tile;
    state->inst_gauss = inst_gauss;
    state->tile_range = reinterpret_cast<const uint32_t *>(ranges);
    state->tile_work = tile_work;
    return OMNIGS_OK;
}

omnigs_status omnigs_backward(const omnigs_gaussians *g, const omnigs_camera *cam, const omnigs_settings *s,
                              const omnigs_state *state, const omnigs_image_out *fwd, const float *dL_dimage,
                              omnigs_grads *grads, omnigs_allocator alloc, void *stream) {
    omnigs_status rc;
    if ((rc = check_gaussians(g)) != OMNIGS_OK) return rc;
    if ((rc = check_camera(cam)) != OMNIGS_OK) return rc;
    if ((rc = check_settings(s)) != OMNIGS_OK) return rc;
    if (!alloc.alloc) return fail(OMNIGS_ERR_INVALID, "allocator callback is NULL");
    if (!state || !fwd || !fwd->final_T || !fwd->n_contrib || !dL_dimage || !grads)
        return fail(OMNIGS_ERR_INVALID, "a state, forward-output, cotangent or gradient pointer is NULL");
    if (g->n > 0 && (!grads->dmeans || !grads->dscales || !grads->dquats || !grads->dopacities || !grads->dsh ||
                     !grads->dscreen))
        return fail(OMNIGS_ERR_INVALID, "a gradient output pointer is NULL");
    if (g->n > 0 && reinterpret_cast<uintptr_t>(grads->dquats) % 16 != 0)
        return fail(OMNIGS_ERR_INVALID, "dquats must be 16-byte aligned");
    if (state->n != g->n || state->width != cam->width || state->height != cam->height)
        return fail(OMNIGS_ERR_INVALID, "state does not match the Gaussians / camera");
    if (g->n > 0 && (!state->records || !state->n_tiles || !state->inst_gauss || !state->tile_range ||
                     !state->tile_work))
        return fail(OMNIGS_ERR_INVALID, "state buffers are NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t n = g->n;
    if (n == 0) return OMNIGS_OK;
    const ProjectArgs pa = make_project_args(g, cam, s);
    const uint32_t ntiles = (uint32_t)(pa.tiles_x * pa.tiles_y);
    Arena a;
    a.take<float>((size_t)n * kAcc);
    a.take<uint32_t>(ntiles);
    if ((rc = alloc_arena(alloc, a.off, OMNIGS_MEM_SCRATCH, a, "gradient accumulators")) != OMNIGS_OK) return rc;
    float *acc = a.take<float>((size_t)n * kAcc);
    uint32_t *order = a.take<uint32_t>(ntiles);
    const auto *rec = static_cast<const BlendRecord *>(state->records);
    const auto *ranges = reinterpret_cast<const uint2 *>(state->tile_range);
    {
        StageTimer t(st, kStBwdClear);
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(acc), 0u, n * kAcc, st));
    }
    const FrameGeom f{cam->width, cam->height, pa.tiles_x, pa.tiles_y, 0u};
    {
        StageTimer t(st, kStTileOrder);
        HIP_TRY(launch_tile_order(ranges, state->tile_work, ntiles, order, st));
    }
    {
        StageTimer t(st, kStBlendBwd);
        HIP_TRY(launch_blend_backward(f, rec, state->inst_gauss, ranges, make_blend_settings(s), fwd->final_T,
                                      fwd->n_contrib, dL_dimage, acc, order, st));
    }
    {
        StageTimer t(st, kStProjectBwd);
        HIP_TRY(launch_project_backward(pa, state->n_tiles, acc, *grads, st));
    }
    return OMNIGS_OK;
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

omnigs_status omnigs_forward_batch(const omnigs_gaussians *g, const omnigs_camera *cams, int32_t batch,
                                   const omnigs_settings *s, omnigs_allocator alloc, omnigs_image_out *outs,
                                   int64_t instance_capacity, int32_t *overflow, int64_t *n_instances,
                                   void *stream) {
    omnigs_status rc;
    if (n_instances) *n_instances = -1;
    if ((rc = check_gaussians(g)) != OMNIGS_OK) return rc;
    if ((rc = check_settings(s)) != OMNIGS_OK) return rc;
    if (batch < 1 || batch > kMaxBatch) return fail(OMNIGS_ERR_INVALID, "batch %d not in [1, %d]", batch, kMaxBatch);
    if (!cams || !outs) return fail(OMNIGS_ERR_INVALID, "cameras or outputs is NULL");
    if (!alloc.alloc) return fail(OMNIGS_ERR_INVALID, "allocator callback is NULL");
    if (instance_capacity < 0 || instance_capacity >= (int64_t(1) << 32))
        return fail(OMNIGS_ERR_INVALID, "instance_capacity %lld out of range", (long long)instance_capacity);
    const int64_t n = g->n;
    const int64_t nrec = n * batch;  // record b * n + i: camera b, Gaussian i
    if (nrec >= (int64_t(1) << 32) - 1) return fail(OMNIGS_ERR_INVALID, "batch * n must stay below 2^32");
    uint64_t total_tiles = 0;
    FrameGeom frames[kMaxBatch];
    CamTable ct{};
    ct.count = batch;
    EmitFrames ef{};
    ef.n_per = n > 0 ? n : 1;
    ef.count = batch;
    for (int b = 0; b < batch; ++b) {
        if ((rc = check_camera(&cams[b])) != OMNIGS_OK) return rc;
        if (!outs[b].image || !outs[b].final_T || !outs[b].n_contrib)
            return fail(OMNIGS_ERR_INVALID, "output pointer of camera %d is NULL", b);
        const ProjectArgs pb = make_project_args(g, &cams[b], s);
        CamGeom &cg = ct.c[b];
        for (int k = 0; k < 9; ++k) cg.R[k] = pb.R[k];
        for (int k = 0; k < 3; ++k) {
            cg.t[k] = pb.t[k];
            cg.campos[k] = pb.campos[k];
        }
        cg.width = pb.width;
        cg.height = pb.height;
        cg.tiles_x = pb.tiles_x;
        cg.tiles_y = pb.tiles_y;
        frames[b] = FrameGeom{pb.width, pb.height, pb.tiles_x, pb.tiles_y, (uint32_t)total_tiles};
        ef.tiles_x[b] = pb.tiles_x;
        ef.tile_base[b] = (uint32_t)total_tiles;
        total_tiles += (uint64_t)pb.tiles_x * pb.tiles_y;
    }
    // the last id is kept free so that bits_for always has room
    if (total_tiles >= (uint64_t(1) << 31)) return fail(OMNIGS_ERR_INVALID, "too many tiles in the batch");
    const ProjectArgs pa = make_project_args(g, &cams[0], s);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t ntiles = (uint32_t)total_tiles;

    // per-record buffers (all scratch: no backward state is kept)
    Arena ra;
    GeomState gst;
    GeomScratch gs;
    auto carve_geom = [&](Arena &a) {
        gst.carve(a, nrec);
        gs.carve(a, nrec);
    };
    carve_geom(ra);
    if ((rc = alloc_arena(alloc, ra.off, OMNIGS_MEM_SCRATCH, ra, "per-record scratch")) != OMNIGS_OK) return rc;
    carve_geom(ra);
    if (overflow) HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(overflow), 0u, 1, st));
    {
        StageTimer t(st, kStProject);
        HIP_TRY(launch_project_batch(pa, ct, gst.rec, gs.depth_key, gst.n_tiles, gst.rect, st));
    }
    {
        StageTimer t(st, kStDepthSort);
        HIP_TRY(launch_iota(gs.iota, nrec, st));
        HIP_TRY(radix_sort_pairs(gs.depth_key, gs.iota, gs.keys_tmp, gs.vals_tmp, gs.keys_sorted, gst.order, nrec,
                                 32, gs.sort_tmp, st));
    }
    uint32_t *m_dev = gs.offs + nrec;
    {
        StageTimer t(st, kStEmitCount);
        HIP_TRY(scan_exclusive(gst.n_tiles, gs.offs, nrec, m_dev, gs.scan_tmp, st, gst.order));
    }
    int64_t cap = instance_capacity;
    if (cap == 0) {
        uint32_t m32 = 0;
        HIP_TRY(hipMemcpyAsync(&m32, m_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        cap = m32;
        if (n_instances) *n_instances = m32;
    }
    const int bits = bits_for(total_tiles);
    const int passes = (bits + 7) / 8;
    const size_t mc = (size_t)(cap > 0 ? cap : 1);
    Arena ia;
    uint32_t *inst_tile, *inst_gauss, *tmp_tile, *tmp_gauss, *part, *order;
    uint2 *ranges;
    void *sort_tmp;
    auto carve_inst = [&](Arena &a) {
        inst_tile = a.take<uint32_t>(mc);
        inst_gauss = a.take<uint32_t>(mc);
        tmp_tile = a.take<uint32_t>(mc);
        tmp_gauss = a.take<uint32_t>(mc);
        sort_tmp = a.take_bytes(sort_scratch_bytes((int64_t)mc));
        part = a.take<uint32_t>((size_t)emit_blocks((uint64_t)cap) + 1);
        ranges = a.take<uint2>(ntiles);
        order = a.take<uint32_t>(ntiles);
    };
    carve_inst(ia);
    if ((rc = alloc_arena(alloc, ia.off, OMNIGS_MEM_SCRATCH, ia, "instance lists")) != OMNIGS_OK) return rc;
    carve_inst(ia);
    // with a capacity, the counts the kernels use are min(M, capacity),
    // read on the device
    const uint32_t *count_dev = instance_capacity > 0 ? m_dev : nullptr;
    {
        StageTimer t(st, kStEmit);
        const bool odd = passes % 2;
        HIP_TRY(launch_emit(gst.order, gst.n_tiles, gst.rect, gs.offs, nrec, part, m_dev, ef, (uint64_t)cap,
                            odd ? tmp_tile : inst_tile, odd ? tmp_gauss : inst_gauss, overflow, st));
    }
    {
        StageTimer t(st, kStTileSort);
        const bool odd = passes % 2;
        HIP_TRY(radix_sort_pairs(odd ? tmp_tile : inst_tile, odd ? tmp_gauss : inst_gauss, tmp_tile, tmp_gauss,
                                 inst_tile, inst_gauss, cap, bits, sort_tmp, st, count_dev));
    }
    {
        StageTimer t(st, kStRanges);
        HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(ranges), 0u, 2 * (int64_t)ntiles, st));
        HIP_TRY(launch_tile_ranges(inst_tile, m_dev, (uint64_t)cap, ranges, ntiles, st));
    }
    {
        StageTimer t(st, kStTileOrder);
        HIP_TRY(launch_tile_order(ranges, nullptr, ntiles, order, st));
    }
    {
        StageTimer t(st, kStBlendFwd);
        HIP_TRY(launch_blend_forward_frames(frames, outs, batch, gst.rec, inst_gauss, ranges, make_blend_settings(s),
                                            order, ntiles, st));
    }
    return OMNIGS_OK;
}

omnigs_status omnigs_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on != 0;
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
