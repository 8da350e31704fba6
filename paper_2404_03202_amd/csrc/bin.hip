// bin.hip -- second level of the tile binning (Sec. 3.3: one instance per
// (Gaussian, covered tile), each tile's list ordered by t_r).
//
// The first level (sort.hip) leaves, for every super-tile of 8x8 tiles, the
// list of records whose tile rectangle touches it, in depth order.  Here each
// list is cut into chunks of kChunk entries.  The tiles of its super-tile
// that an entry's record covers are a product of covered rows and covered
// columns (its rectangle, columns wrapping across the seam, clipped to the
// super-tile), so per wave 8 row ballots and 8 column ballots give, for each
// of the 64 tiles, the lanes that cover it (the AND of its row's and its
// column's ballots): the tile's instance count and, in the expansion, each
// entry's rank among the chunk's entries that cover the tile, in list
// order.  Counts are laid out per super-tile as [tile][chunk],
// super-tiles one after another, so that one exclusive scan yields at once
// the start of every tile's list (tiles are stored super-tile by super-tile,
// each tile's list contiguous) and the offset of every chunk inside it.
// Every instance is then written once, to its final position: each tile's
// list comes out in depth order, as a stable sort on the tile id would give.
#include "internal.h"

#include <algorithm>

namespace omnigs {
namespace {

constexpr int kChunk = 256;  // super-list entries per chunk (one per thread)
constexpr int kThreads = kChunk;
constexpr int kWaves = kThreads / kWave;
constexpr int kTilesPer = kSuper * kSuper;  // 64 tiles per super-tile
constexpr uint32_t kXcds = 8;  // XCDs of the device, each with its own L2

__device__ inline int find_super_frame(const SuperTable &T, uint32_t s) {
    int f = 0;
    for (int k = 1; k < T.count; ++k)
        if (s >= T.f[k].super_base) f = k;
    return f;
}

// The wave's ballots of covered rows and columns: lane q < 8 receives the
// ballot of row q, lane 8 + q that of column q.  The lanes covering tile
// (k, c) are then rowball(k) & colball(c): a product of rectangles is the
// product of their row and column sets.
__device__ inline uint64_t row_col_ballots(Cover cv, int lane) {
    uint64_t mine = 0ull;
#pragma unroll
    for (int q = 0; q < kSuper; ++q) {
        const uint64_t br = __ballot((cv.rows >> q) & 1u);
        const uint64_t bc = __ballot((cv.cols >> q) & 1u);
        mine = lane == q ? br : mine;
        mine = lane == kSuper + q ? bc : mine;
    }
    return mine;
}

// Position of (super-tile s, tile j, chunk c) in the count layout.
__device__ inline uint64_t layout(uint32_t choff_s, uint32_t nch_s, int j, uint32_t c) {
    return (uint64_t)kTilesPer * choff_s + (uint64_t)j * nch_s + c;
}

// Chunks of each super-tile's list.
__global__ __launch_bounds__(256) void k_bin_chunks(const uint2 *sranges, uint32_t n_super, uint32_t *nch) {
    const uint32_t s = blockIdx.x * 256u + threadIdx.x;
    if (s >= n_super) return;
    const uint32_t len = sranges[s].y - sranges[s].x;
    nch[s] = (len + kChunk - 1) / kChunk;
}

// desc[k] = super-tile of chunk k: the last s with choff[s] <= k (super-tiles
// without chunks share their offset with the next one), one thread per chunk.
__global__ __launch_bounds__(256) void k_bin_desc(const uint32_t *choff, uint32_t n_super, uint64_t max_chunks,
                                                  uint32_t *desc) {
    const uint64_t k = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (k >= max_chunks || k >= choff[n_super]) return;
    uint32_t lo = 0, hi = n_super;  // choff[lo] <= k < choff[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (choff[mid] <= k) lo = mid; else hi = mid;
    }
    desc[k] = lo;
}

__global__ __launch_bounds__(kThreads) void k_bin_count(SuperTable T, const uint2 *rect, const uint32_t *skeys,
                                                        const uint32_t *sinst_gauss,
                                                        const uint2 *sranges, const uint32_t *choff,
                                                        const uint32_t *nch, const uint32_t *desc, uint32_t n_super,
                                                        uint32_t *counts) {
    __shared__ uint64_t rc[kWaves][2 * kSuper];
    const uint32_t k = blockIdx.x;
    const uint32_t K = choff[n_super];  // chunks in all (device)
    const int w = threadIdx.x / kWave, lane = __lane_id();
    if (k >= K) {
        // slots past the last chunk: zero, so that the scan over the whole
        // (capacity-sized) layout leaves every valid position exact
        if (threadIdx.x < kTilesPer) counts[(uint64_t)kTilesPer * k + threadIdx.x] = 0u;
        return;
    }
    const uint32_t s = desc[k], o = choff[s], n = nch[s], c = k - o;
    const SuperFrame &F = T.f[find_super_frame(T, s)];
    const uint32_t ls = s - F.super_base;
    const int sx = (int)(ls % (uint32_t)F.super_x), sy = (int)(ls / (uint32_t)F.super_x);
    const uint32_t e = sranges[s].x + c * kChunk + threadIdx.x;
    Cover cv{0u, 0u};
    if (e < sranges[s].y) cv = skeys ? cover_from_key(skeys[e]) : cover_of(rect[sinst_gauss[e]], F.tiles_x, sx, sy);
    const uint64_t b = row_col_ballots(cv, lane);
    if (lane < 2 * kSuper) rc[w][lane] = b;
    __syncthreads();
    if (threadIdx.x < kTilesPer) {
        const int j = threadIdx.x;
        uint32_t t = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) t += (uint32_t)__popcll(rc[q][j / kSuper] & rc[q][kSuper + j % kSuper]);
        counts[layout(o, n, j, c)] = t;
    }
}

// Chunks, chunk offsets and chunk owners in one workgroup, for fewer than
// kPlanMax super-tiles: nch[s], choff[s] (exclusive scan, choff[n_super]
// the total) and desc[k] = s for every chunk k < min(total, max_chunks)
// with choff[s] <= k < choff[s + 1], as k_bin_chunks, the scan and
// k_bin_desc give them.
constexpr int kPlanThreads = 1024;
constexpr int kPlanPer = 8;  // super-tiles per thread
constexpr uint32_t kPlanMax = kPlanThreads * kPlanPer;
__global__ __launch_bounds__(kPlanThreads) void k_bin_plan(const uint2 *sranges, uint32_t n_super,
                                                          uint64_t max_chunks, uint32_t *nch, uint32_t *choff,
                                                          uint32_t *desc) {
    __shared__ uint32_t s_off[kPlanMax];
    __shared__ uint32_t wave_tot[kPlanThreads / kWave];
    uint32_t v[kPlanPer], sum = 0;
#pragma unroll
    for (int q = 0; q < kPlanPer; ++q) {
        const uint32_t sidx = threadIdx.x * kPlanPer + q;
        v[q] = 0;
        if (sidx < n_super) {
            const uint2 r = sranges[sidx];
            v[q] = (r.y - r.x + kChunk - 1) / kChunk;
            nch[sidx] = v[q];
        }
        sum += v[q];
    }
    const int lane = __lane_id(), wv = threadIdx.x / kWave;
    uint32_t x = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) wave_tot[wv] = x;
    __syncthreads();
    uint32_t run = x - sum;
    for (int k = 0; k < wv; ++k) run += wave_tot[k];
    // n_super < kPlanMax: the slot n_super (the total) lies in some thread's
    // range, and every v past n_super is zero
#pragma unroll
    for (int q = 0; q < kPlanPer; ++q) {
        const uint32_t sidx = threadIdx.x * kPlanPer + q;
        if (sidx <= n_super) {
            s_off[sidx] = run;
            choff[sidx] = run;
        }
        run += v[q];
    }
    __syncthreads();
    // chunk owners: wave w writes the chunks of super-tiles w, w + 16, ...,
    // its lanes along each run [choff[s], choff[s + 1]) (a search per chunk
    // took 27 us at 35k chunks)
    constexpr int kPlanWaves = kPlanThreads / kWave;
    for (uint32_t sidx = wv; sidx < n_super; sidx += kPlanWaves) {
        const uint64_t a = s_off[sidx], b = s_off[sidx + 1];
        const uint64_t e = b < max_chunks ? b : max_chunks;
        for (uint64_t k = a + lane; k < e; k += kWave) desc[k] = sidx;
    }
}

// [start, end) of every tile, from the scanned counts.
__global__ __launch_bounds__(256) void k_bin_ranges(SuperTable T, uint32_t n_super, const uint32_t *choff,
                                                    const uint32_t *nch, const uint32_t *scanned, uint64_t inst_cap,
                                                    uint2 *ranges) {
    const uint64_t id = (uint64_t)blockIdx.x * 256u + threadIdx.x;
    if (id >= (uint64_t)n_super * kTilesPer) return;
    const uint32_t s = (uint32_t)(id / kTilesPer);
    const int j = (int)(id % kTilesPer);
    const SuperFrame &F = T.f[find_super_frame(T, s)];
    const uint32_t ls = s - F.super_base;
    const int tx = (int)(ls % (uint32_t)F.super_x) * kSuper + j % kSuper;
    const int ty = (int)(ls / (uint32_t)F.super_x) * kSuper + j / kSuper;
    if (tx >= F.tiles_x || ty >= F.tiles_y) return;
    const uint32_t o = choff[s], n = nch[s];
    uint64_t a = scanned[layout(o, n, j, 0)], b = scanned[layout(o, n, j + 1, 0)];
    a = a < inst_cap ? a : inst_cap;
    b = b < inst_cap ? b : inst_cap;
    ranges[F.tile_base + (uint32_t)ty * (uint32_t)F.tiles_x + (uint32_t)tx] = make_uint2((uint32_t)a, (uint32_t)b);
}

// Every instance of the chunk to its final position.
__global__ __launch_bounds__(kThreads) void k_bin_expand(SuperTable T, const uint2 *rect, const uint32_t *skeys,
                                                         const uint32_t *sinst_gauss,
                                                         const uint2 *sranges, const uint32_t *choff,
                                                         const uint32_t *nch, const uint32_t *desc, uint32_t n_super,
                                                         const uint32_t *scanned, uint64_t inst_cap,
                                                         uint32_t *inst_gauss, int32_t *overflow,
                                                         const uint32_t *fault, const uint2 *ranges,
                                                         uint32_t order_tiles, uint32_t *order) {
    __shared__ union {
        struct {
            uint64_t rc[kWaves][2 * kSuper];
            uint32_t wpre[kWaves][kTilesPer];
        } e;
        TileOrderShared o;
    } sh;
    auto &rc = sh.e.rc;
    auto &wpre = sh.e.wpre;
    // the first kXcds workgroups take no chunk: workgroup 0 (dispatched
    // first, so it runs beside the expansion) writes the blend's launch order
    // from the tile ranges when asked; workgroup 1 merges the fault word: a
    // lookback wait of the sorts or scans before this kernel that gave up
    // marks the overflow word too (bit 1), so that a caller who reads nothing
    // back but that word still sees it
    if (blockIdx.x < kXcds) {
        if (blockIdx.x == 0 && order && order_tiles > 0)
            tile_order_block<kThreads>(ranges, nullptr, order_tiles, order, sh.o);
        if (blockIdx.x == 1 && threadIdx.x == 0 && fault && overflow && *fault) atomicOr(overflow, 2);
        return;
    }
    // workgroups go to the XCDs in turn (workgroup b to XCD b mod 8): XCD x
    // takes the chunks [x per, (x + 1) per) in order, so the chunks that write
    // adjacent pieces of a tile's list run on one XCD and their partial cache
    // lines meet in its L2 (after the kXcds leading workgroups, the grid is a
    // multiple of 8 and covers 8 per)
    const uint32_t wg = blockIdx.x - kXcds;
    const uint32_t total = choff[n_super], per = (total + kXcds - 1) / kXcds;
    const uint32_t k = (wg % kXcds) * per + wg / kXcds;
    if (wg / kXcds >= per || k >= total) return;
    const int w = threadIdx.x / kWave, lane = __lane_id();
    const uint32_t s = desc[k], o = choff[s], n = nch[s], c = k - o;
    const SuperFrame &F = T.f[find_super_frame(T, s)];
    const uint32_t ls = s - F.super_base;
    const int sx = (int)(ls % (uint32_t)F.super_x), sy = (int)(ls / (uint32_t)F.super_x);
    const uint32_t e = sranges[s].x + c * kChunk + threadIdx.x;
    Cover cv{0u, 0u};
    uint32_t g = 0;
    if (e < sranges[s].y) {
        g = sinst_gauss[e];
        cv = skeys ? cover_from_key(skeys[e]) : cover_of(rect[g], F.tiles_x, sx, sy);
    }
    const uint64_t b = row_col_ballots(cv, lane);
    if (lane < 2 * kSuper) rc[w][lane] = b;
    __syncthreads();
    if (threadIdx.x < kTilesPer) {
        // start of this chunk's instances in tile j, plus the entries of the
        // earlier waves that cover the tile
        const int j = threadIdx.x;
        uint32_t run = scanned[layout(o, n, j, c)];
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
            wpre[q][j] = run;
            run += (uint32_t)__popcll(rc[q][j / kSuper] & rc[q][kSuper + j % kSuper]);
        }
    }
    __syncthreads();
    // tile by tile (uniform loops over the wave's covered rows and columns);
    // the lanes of one tile write consecutive positions
    const uint64_t below = (1ull << lane) - 1ull;
    bool dropped = false;
    for (int r = 0; r < kSuper; ++r) {
        const uint64_t br = rc[w][r];
        if (br == 0ull) continue;  // uniform
        for (int q = 0; q < kSuper; ++q) {
            const uint64_t bt = br & rc[w][kSuper + q];
            if (bt == 0ull) continue;  // uniform
            if ((bt >> lane) & 1ull) {
                const uint64_t pos = (uint64_t)wpre[w][r * kSuper + q] + (uint64_t)__popcll(bt & below);
                if (pos < inst_cap) inst_gauss[pos] = g;
                else dropped = true;
            }
        }
    }
    if (dropped && overflow) atomicOr(overflow, 1);
}

int64_t blocks_for(int64_t n, int64_t per) { return (n + per - 1) / per; }

uint64_t max_chunks(uint64_t super_cap, uint32_t n_super_total) {
    return (super_cap + kChunk - 1) / kChunk + n_super_total;
}

}  // namespace

// Scratch layout: nch | choff | desc | counts | scanned | scan scratch of the
// chunk offsets | scan scratch of the counts (each 256-byte aligned).
struct BinLayout {
    uint32_t *nch, *choff, *desc, *counts, *scanned;
    void *scan_chunks, *scan_counts;
    size_t bytes;
    BinLayout(void *scratch, uint64_t super_cap, uint32_t n_super_total) {
        const uint64_t K = max_chunks(super_cap, n_super_total);
        const uint64_t cells = (uint64_t)kTilesPer * K;
        auto al = [](uint64_t b) { return (size_t)((b + 255) & ~(uint64_t)255); };
        char *base = static_cast<char *>(scratch), *p = base;
        auto take = [&](size_t b) {
            char *q = p;
            p += al(b);
            return q;
        };
        nch = reinterpret_cast<uint32_t *>(take(4ull * n_super_total));
        choff = reinterpret_cast<uint32_t *>(take(4ull * (n_super_total + 1)));
        desc = reinterpret_cast<uint32_t *>(take(4ull * K));
        counts = reinterpret_cast<uint32_t *>(take(4ull * cells));
        scanned = reinterpret_cast<uint32_t *>(take(4ull * (cells + 1)));
        scan_chunks = take(scan_scratch_bytes((int64_t)n_super_total));
        scan_counts = take(scan_scratch_bytes((int64_t)cells));
        bytes = (size_t)(p - base) + 256;
    }
};

size_t binning_scratch_bytes(uint64_t super_cap, uint32_t n_super_total) {
    return BinLayout(nullptr, super_cap, n_super_total).bytes;
}

void binning_clear(void *scratch, uint64_t super_cap, uint32_t n_super_total, ClearList &L) {
    if (n_super_total == 0) return;
    const BinLayout B(scratch, super_cap, n_super_total);
    const uint64_t cells = (uint64_t)kTilesPer * max_chunks(super_cap, n_super_total);
    L.add(B.scan_counts, scan_clear_words((int64_t)cells));
}

hipError_t launch_binning(const SuperTable &T, uint32_t n_super_total, const uint2 *rect, const uint32_t *skeys,
                          const uint32_t *sinst_gauss, const uint2 *sranges, uint64_t super_cap, uint64_t inst_cap,
                          void *scratch, uint2 *ranges,
                          uint32_t *inst_gauss, int32_t *overflow, hipStream_t st, bool cleared,
                          uint32_t *fault, uint32_t *order, uint32_t order_tiles) {
    if (n_super_total == 0) {
        // no lists: every tile's range is empty and any order is longest first
        if (order && order_tiles > 0) {
            hipError_t e = launch_tile_order(ranges, nullptr, order_tiles, order, st);
            if (e != hipSuccess) return e;
        }
        return overflow && fault ? launch_merge_fault(fault, overflow, st) : hipSuccess;
    }
    const uint64_t K = max_chunks(super_cap, n_super_total);
    const uint64_t cells = (uint64_t)kTilesPer * K;
    const BinLayout B(scratch, super_cap, n_super_total);
    const unsigned sb = (unsigned)blocks_for(n_super_total, 256);
    hipError_t e;
    // the one-workgroup plan goes with the cover keys, so that the knob that
    // turns those off (for tests) exercises the three-kernel path as well
    if (skeys && n_super_total < kPlanMax) {
        hipLaunchKernelGGL(k_bin_plan, dim3(1), dim3(kPlanThreads), 0, st, sranges, n_super_total, K, B.nch, B.choff,
                           B.desc);
    } else {
        hipLaunchKernelGGL(k_bin_chunks, dim3(sb), dim3(256), 0, st, sranges, n_super_total, B.nch);
        e = scan_exclusive(B.nch, B.choff, n_super_total, B.choff + n_super_total, B.scan_chunks, st, nullptr, false,
                           fault);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_bin_desc, dim3((unsigned)blocks_for((int64_t)K, 256)), dim3(256), 0, st, B.choff,
                           n_super_total, K, B.desc);
    }
    hipLaunchKernelGGL(k_bin_count, dim3((unsigned)K), dim3(kThreads), 0, st, T, rect, skeys, sinst_gauss, sranges,
                       B.choff, B.nch, B.desc, n_super_total, B.counts);
    e = scan_exclusive(B.counts, B.scanned, (int64_t)cells, B.scanned + cells, B.scan_counts, st, nullptr, cleared,
                       fault);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_ranges, dim3((unsigned)blocks_for((int64_t)n_super_total * kTilesPer, 256)), dim3(256), 0,
                       st, T, n_super_total, B.choff, B.nch, B.scanned, inst_cap, ranges);
    hipLaunchKernelGGL(k_bin_expand, dim3((unsigned)(kXcds + (K + kXcds - 1) / kXcds * kXcds)), dim3(kThreads), 0, st,
                       T, rect, skeys, sinst_gauss, sranges, B.choff, B.nch, B.desc, n_super_total, B.scanned, inst_cap,
                       inst_gauss, overflow, fault, ranges, order_tiles, order);
    return hipGetLastError();
}

namespace {
__global__ void k_merge_fault(const uint32_t *fault, int32_t *overflow) {
    if (*fault) *overflow |= 2;
}
}  // namespace

hipError_t launch_merge_fault(const uint32_t *fault, int32_t *overflow, hipStream_t st) {
    hipLaunchKernelGGL(k_merge_fault, dim3(1), dim3(1), 0, st, fault, overflow);
    return hipGetLastError();
}

}  // namespace omnigs
