// sort.hip -- binning of Gaussian instances into 16x16 tiles (Sec. 3.3: "each
// tile counts the 2D Gaussians whose radius of influence covers this tile,
// generating one instance per influence"), ordered by distance t_r inside
// each tile (Sec. 3.3: ERP sorts by t_r, not t_z).
//
// Instead of one wide (tile | depth) key sort over all M instances, the
// order is built in two narrow stable sorts:
//   1. the N Gaussians are sorted by the float bits of t_r (4 passes over N);
//   2. instances are emitted in that depth order (a scan of tiles-per-
//      Gaussian in depth order gives each Gaussian its output range; every
//      block writes a fixed span of consecutive outputs, coalesced), then
//      stably radix-sorted on the tile id alone (ceil(log2 tiles / 8)
//      passes over M).
// The result is each tile's list in (t_r, Gaussian id) order, identical to a
// sort on (tile, t_r, id), with ~4x less traffic than a 6-pass 64-bit key
// sort over M.
//
// The LSD passes use 8-bit digits.  A pass is: per-block digit histogram,
// exclusive scan of the [digit][block] count matrix, and a scatter in which
// each wave ranks its keys with ballot-based match (8 ballots per key, wave64),
// the block places keys in LDS in digit order, and writes them out as
// contiguous per-digit runs.
#include "internal.h"

namespace omnigs {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
#ifndef OMNIGS_SORT_ITEMS
#define OMNIGS_SORT_ITEMS 8
#endif
constexpr int kItems = OMNIGS_SORT_ITEMS;   // keys per thread per pass
constexpr int kTileKeys = kThreads * kItems;  // keys per block
constexpr int kRadixBits = 8;
constexpr int kBins = 1 << kRadixBits;
constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;
constexpr int kEmitItems = 8;
constexpr int kEmitSpan = kThreads * kEmitItems;  // outputs per emit block

__device__ inline uint64_t lanemask_lt() { return (1ull << __lane_id()) - 1ull; }

// Lanes of the wave whose `valid` is set and whose digit equals this lane's.
__device__ inline uint64_t match_digit(uint32_t d, int bits, bool valid) {
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
        const bool set = (d >> b) & 1u;
        const uint64_t m = __ballot(set);
        peers &= set ? m : ~m;
    }
    return peers;
}

// Block-wide exclusive scan of one u32 per thread (256 threads); returns the
// prefix and writes the block total to *total (LDS).
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *wave_tot, uint32_t *total) {
    const int lane = __lane_id(), w = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) wave_tot[w] = x;
    __syncthreads();
    uint32_t base = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        const uint32_t t = wave_tot[k];
        base += (k < w) ? t : 0u;
        all += t;
    }
    if (threadIdx.x == 0) *total = all;
    __syncthreads();
    return base + x - v;
}

// ---------------------------------------------------------------- radix pass
// Element count of a sort: n, or min(n, *n_dev) when counted on the device.
__device__ inline int64_t sort_count(int64_t n, const uint32_t *n_dev) {
    if (!n_dev) return n;
    const int64_t m = *n_dev;
    return m < n ? m : n;
}

__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t *keys, int64_t n_max, const uint32_t *n_dev,
                                                          int shift, int bits, uint32_t *counts, int nblocks) {
    __shared__ uint32_t hist[kWaves][kBins];
    const int64_t n = sort_count(n_max, n_dev);
    const int w = threadIdx.x / kWave, lane = __lane_id();
    for (int k = threadIdx.x; k < kWaves * kBins; k += kThreads) (&hist[0][0])[k] = 0;
    __syncthreads();
    const uint32_t mask = (1u << bits) - 1u;
    const int64_t base = (int64_t)blockIdx.x * kTileKeys + (int64_t)w * (kItems * kWave);
#pragma unroll 4
    for (int it = 0; it < kItems; ++it) {
        const int64_t idx = base + it * kWave + lane;
        const bool valid = idx < n;
        const uint32_t d = valid ? (keys[idx] >> shift) & mask : 0u;
        const uint64_t peers = match_digit(d, bits, valid);
        if (valid && (peers & lanemask_lt()) == 0) hist[w][d] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kBins; d += kThreads) {
        if (d <= (int)mask) {
            uint32_t s = 0;
            for (int k = 0; k < kWaves; ++k) s += hist[k][d];
            counts[(int64_t)d * nblocks + blockIdx.x] = s;
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_radix_scatter(const uint32_t *keys_in, const uint32_t *vals_in,
                                                             uint32_t *keys_out, uint32_t *vals_out, int64_t n_max,
                                                             const uint32_t *n_dev, int shift, int bits,
                                                             const uint32_t *offsets, int nblocks) {
    __shared__ uint32_t s_keys[kTileKeys];
    __shared__ uint32_t s_vals[kTileKeys];
    __shared__ uint32_t cnt[kWaves][kBins];
    __shared__ uint32_t digit_start[kBins];
    __shared__ uint32_t gbase[kBins];
    __shared__ uint32_t wave_tot[kWaves];
    __shared__ uint32_t total;
    const int64_t n = sort_count(n_max, n_dev);
    const int w = threadIdx.x / kWave, lane = __lane_id();
    const uint32_t mask = (1u << bits) - 1u;
    const int64_t block0 = (int64_t)blockIdx.x * kTileKeys;
    const int64_t base = block0 + (int64_t)w * (kItems * kWave);
    for (int k = threadIdx.x; k < kWaves * kBins; k += kThreads) (&cnt[0][0])[k] = 0;
    __syncthreads();
    uint32_t key[kItems], val[kItems], rank[kItems];
    // keys past n get the largest digit: they sort last in the block and are
    // never written out
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int64_t idx = base + it * kWave + lane;
        const bool valid = idx < n;
        key[it] = valid ? keys_in[idx] : 0xffffffffu;
        val[it] = valid ? vals_in[idx] : 0u;
    }
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int64_t idx = base + it * kWave + lane;
        const uint32_t d = (idx < n) ? (key[it] >> shift) & mask : mask;
        const uint64_t peers = match_digit(d, bits, true);
        const uint32_t before = cnt[w][d];
        rank[it] = before + (uint32_t)__popcll(peers & lanemask_lt());
        if ((peers & lanemask_lt()) == 0) cnt[w][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // digit-major block layout: digit_start[d] + sum of earlier waves' counts
    const int d = threadIdx.x;  // kThreads == kBins
    uint32_t per[kWaves], tot = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        per[k] = cnt[k][d];
        tot += per[k];
    }
    const uint32_t start = block_exclusive_scan(tot, wave_tot, &total);
    digit_start[d] = start;
    {
        uint32_t run = start;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
            cnt[k][d] = run;
            run += per[k];
        }
    }
    if (d <= (int)mask) gbase[d] = offsets[(int64_t)d * nblocks + blockIdx.x] - start;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kItems; ++it) {
        const int64_t idx = base + it * kWave + lane;
        const uint32_t dg = (idx < n) ? (key[it] >> shift) & mask : mask;
        const uint32_t pos = cnt[w][dg] + rank[it];
        s_keys[pos] = key[it];
        s_vals[pos] = val[it];
    }
    __syncthreads();
    int64_t nvalid = n - block0 < kTileKeys ? n - block0 : kTileKeys;
    if (nvalid < 0) nvalid = 0;
    for (int p = threadIdx.x; p < nvalid; p += kThreads) {
        const uint32_t k = s_keys[p];
        const uint32_t dg = (k >> shift) & mask;
        const uint32_t dst = gbase[dg] + (uint32_t)p;
        if (dst < (uint64_t)n) {
            keys_out[dst] = k;
            vals_out[dst] = s_vals[p];
        }
    }
}

// ------------------------------------------------------------------- scans
// Element idx of a scan input: in[idx], or in[gather[idx]] (gathered
// indices past n read as 0).
__device__ inline uint32_t scan_input(const uint32_t *in, const uint32_t *gather, int64_t idx, int64_t n) {
    if (!gather) return in[idx];
    const uint32_t g = gather[idx];
    return g < (uint64_t)n ? in[g] : 0u;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t *in, const uint32_t *gather, int64_t n,
                                                           uint32_t *block_sums) {
    __shared__ uint32_t wave_tot[kWaves];
    __shared__ uint32_t total;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
    uint32_t s = 0;
#pragma unroll
    for (int it = 0; it < kScanItems; ++it) {
        const int64_t idx = base + (int64_t)it * kThreads;
        if (idx < n) s += scan_input(in, gather, idx, n);
    }
    block_exclusive_scan(s, wave_tot, &total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// exclusive scan of a tile with a per-block offset; blocked arrangement:
// thread t owns items [t*kScanItems, (t+1)*kScanItems)
__global__ __launch_bounds__(kThreads) void k_scan_tile(const uint32_t *in, const uint32_t *gather, uint32_t *out,
                                                         int64_t n, const uint32_t *block_offsets,
                                                         uint32_t *grand_total) {
    __shared__ uint32_t wave_tot[kWaves];
    __shared__ uint32_t total;
    __shared__ uint32_t s_data[kScanTile];
    const int64_t block0 = (int64_t)blockIdx.x * kScanTile;
    for (int k = threadIdx.x; k < kScanTile; k += kThreads) {
        const int64_t idx = block0 + k;
        s_data[k] = idx < n ? scan_input(in, gather, idx, n) : 0u;
    }
    __syncthreads();
    uint32_t v[kScanItems], s = 0;
#pragma unroll
    for (int it = 0; it < kScanItems; ++it) {
        v[it] = s_data[threadIdx.x * kScanItems + it];
        s += v[it];
    }
    uint32_t run = block_exclusive_scan(s, wave_tot, &total);
    if (block_offsets) run += block_offsets[blockIdx.x];
#pragma unroll
    for (int it = 0; it < kScanItems; ++it) {
        s_data[threadIdx.x * kScanItems + it] = run;
        run += v[it];
    }
    if (grand_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kThreads - 1) *grand_total = run;
    __syncthreads();
    for (int k = threadIdx.x; k < kScanTile; k += kThreads) {
        const int64_t idx = block0 + k;
        if (idx < n) out[idx] = s_data[k];
    }
}

// ---------------------------------------------------------------- emission
// Entries are emitted in depth order: rank r of the depth order owns the
// output range [offs[r], offs[r] + count(r)), count = tiles or super-tiles of
// its rectangle (the scan behind offs used the same count).  Every emit block writes a
// fixed span of kEmitSpan consecutive outputs, whatever the tile counts of the
// Gaussians behind them (the nearest Gaussians, which come first, cover up to
// thousands of tiles each).  part[b] = the rank owning output b * kEmitSpan.
__global__ __launch_bounds__(kThreads) void k_emit_partition(const uint32_t *order, const uint32_t *n_tiles,
                                                              const uint32_t *offs, int64_t n,
                                                              uint64_t part_blocks, uint32_t *part) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= n) return;
    const uint32_t g = order[r];
    const uint32_t c = g < (uint64_t)n ? n_tiles[g] : 0u;
    if (c == 0) return;
    const uint64_t o = offs[r];
    const uint64_t b1 = (o + c - 1) / kEmitSpan;
    for (uint64_t b = (o + kEmitSpan - 1) / kEmitSpan; b <= b1 && b < part_blocks; ++b) part[b] = (uint32_t)r;
}

__global__ __launch_bounds__(kThreads) void k_emit(const uint32_t *order, const uint32_t *n_tiles, const uint2 *rect,
                                                    const uint32_t *offs, int64_t n, const uint32_t *part,
                                                    const uint32_t *m_dev, EmitFrames F, uint64_t capacity,
                                                    uint32_t *inst_tile, uint32_t *inst_gauss, int32_t *overflow) {
    __shared__ uint32_t s_off[kEmitSpan + 1];
    __shared__ uint32_t s_gid[kEmitSpan + 1];
    __shared__ uint2 s_rect[kEmitSpan + 1];
    __shared__ uint8_t s_cam[kEmitSpan + 1];
    const uint64_t M = *m_dev;
    if (blockIdx.x == 0 && threadIdx.x == 0 && M > capacity && overflow) *overflow = 1;
    const uint64_t j0 = (uint64_t)blockIdx.x * kEmitSpan;
    if (j0 >= M || j0 >= capacity) return;
    // spans that start below min(M, capacity): the grid covers the capacity,
    // and part[] is written for exactly these
    uint64_t nblocks = (M + kEmitSpan - 1) / kEmitSpan;
    if (nblocks > gridDim.x) nblocks = gridDim.x;
    const uint32_t r0 = part[blockIdx.x];
    // ranks of this span: r0 .. r1 (each visible rank owns >= 1 output, so a
    // span of kEmitSpan outputs touches at most kEmitSpan + 1 ranks)
    uint64_t r1 = blockIdx.x + 1 < nblocks ? part[blockIdx.x + 1] : (uint64_t)r0 + kEmitSpan;
    if (r1 > (uint64_t)n - 1) r1 = n - 1;
    if (r1 > (uint64_t)r0 + kEmitSpan) r1 = (uint64_t)r0 + kEmitSpan;
    if (r1 < r0) r1 = r0;
    const int cnt = (int)(r1 - r0) + 1;
    for (int i = threadIdx.x; i < cnt; i += kThreads) {
        const uint32_t r = r0 + i;
        const uint32_t g = order[r];
        // camera of record g = b * n_per + i
        const int cam = F.count > 1 && g < (uint64_t)n ? (int)min((int64_t)g / F.n_per, (int64_t)F.count - 1) : 0;
        uint2 rc = (g < (uint64_t)n && n_tiles[g]) ? rect[g] : make_uint2(0, 0);
        if (F.super) rc = super_rect(rc, F.tiles_x[cam]);
        s_off[i] = offs[r];
        s_gid[i] = g;
        s_rect[i] = rc;
        s_cam[i] = (uint8_t)cam;
    }
    __syncthreads();
    uint64_t jend = j0 + kEmitSpan;
    if (jend > M) jend = M;
    if (jend > capacity) jend = capacity;
    for (uint64_t j = j0 + threadIdx.x; j < jend; j += kThreads) {
        // last rank i with s_off[i] <= j
        int lo = 0, hi = cnt;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_off[mid] <= j) lo = mid; else hi = mid;
        }
        const uint32_t k = (uint32_t)(j - s_off[lo]);
        const uint2 rc = s_rect[lo];
        const uint32_t ntx = rc.x >> 16, tx0 = rc.x & 0xffffu, ty0 = rc.y & 0xffffu;
        if (ntx == 0) continue;
        const int cam = s_cam[lo];
        const uint32_t cols = (uint32_t)F.cols[cam];
        const uint32_t ty = ty0 + k / ntx;
        uint32_t tx = tx0 + k % ntx;
        if (tx >= cols) tx -= cols;
        inst_tile[j] = F.base[cam] + ty * cols + tx;
        inst_gauss[j] = s_gid[lo];
    }
}

// [start, end) of every tile from adjacent sorted instances.  Ranges must be
// zeroed beforehand (empty tiles keep [0, 0)).
__global__ __launch_bounds__(kThreads) void k_tile_ranges(const uint32_t *inst_tile, const uint32_t *m_dev,
                                                           uint64_t capacity, uint2 *ranges, uint32_t n_tiles_total) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    uint64_t m = *m_dev;
    if (m > capacity) m = capacity;
    if (i >= m) return;
    const uint32_t t = inst_tile[i];
    if (t >= n_tiles_total) return;
    if (i == 0 || inst_tile[i - 1] != t) ranges[t].x = (uint32_t)i;
    if (i + 1 == m || inst_tile[i + 1] != t) ranges[t].y = (uint32_t)(i + 1);
}

__global__ void k_iota(uint32_t *v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = (uint32_t)i;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

int64_t blocks_for(int64_t n, int64_t per) { return (n + per - 1) / per; }

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
    // block sums of every level, 256-byte aligned
    size_t bytes = 0;
    int64_t m = n;
    while (m > kScanTile) {
        m = blocks_for(m, kScanTile);
        bytes += ((size_t)m * 4 + 255) & ~(size_t)255;
    }
    return bytes + 256;
}

hipError_t scan_exclusive(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total, void *scratch,
                          hipStream_t st, const uint32_t *gather) {
    if (n <= 0) {
        if (total) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, total, 0u, (int64_t)1);
        return hipGetLastError();
    }
    const int64_t nb = blocks_for(n, kScanTile);
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(kThreads), 0, st, in, gather, out, n,
                           (const uint32_t *)nullptr, total);
        return hipGetLastError();
    }
    uint32_t *sums = static_cast<uint32_t *>(scratch);
    void *next = static_cast<char *>(scratch) + (((size_t)nb * 4 + 255) & ~(size_t)255);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kThreads), 0, st, in, gather, n, sums);
    hipError_t e = scan_exclusive(sums, sums, nb, nullptr, next, st, nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nb), dim3(kThreads), 0, st, in, gather, out, n, sums, total);
    return hipGetLastError();
}

size_t sort_scratch_bytes(int64_t n) {
    const int64_t nb = blocks_for(n > 0 ? n : 1, kTileKeys);
    const int64_t cells = nb * kBins;
    return (((size_t)cells * 4 + 255) & ~(size_t)255) * 2 + scan_scratch_bytes(cells);
}

hipError_t radix_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_tmp,
                            uint32_t *vals_tmp, uint32_t *keys_out, uint32_t *vals_out, int64_t n, int bits,
                            void *scratch, hipStream_t st, const uint32_t *n_dev) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = blocks_for(n, kTileKeys);
    const int64_t cells = nb * kBins;
    uint32_t *counts = static_cast<uint32_t *>(scratch);
    uint32_t *offsets = reinterpret_cast<uint32_t *>(static_cast<char *>(scratch) +
                                                      (((size_t)cells * 4 + 255) & ~(size_t)255));
    void *scan_tmp = reinterpret_cast<char *>(offsets) + (((size_t)cells * 4 + 255) & ~(size_t)255);
    if (bits < 1) bits = 1;
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    // ping-pong so that the last pass lands in keys_out / vals_out
    const uint32_t *src_k = keys_in, *src_v = vals_in;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kRadixBits;
        const int pbits = (bits - shift) < kRadixBits ? (bits - shift) : kRadixBits;
        const bool last = (p == passes - 1);
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        uint32_t *dk = to_out ? keys_out : keys_tmp;
        uint32_t *dv = to_out ? vals_out : vals_tmp;
        (void)last;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kThreads), 0, st, src_k, n, n_dev, shift, pbits,
                           counts, (int)nb);
        // only (1 << pbits) digit rows are used: scan that prefix of the matrix
        hipError_t e = scan_exclusive(counts, offsets, (int64_t)(1 << pbits) * nb, nullptr, scan_tmp, st, nullptr);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kThreads), 0, st, src_k, src_v, dk, dv, n,
                           n_dev, shift, pbits, offsets, (int)nb);
        src_k = dk;
        src_v = dv;
    }
    return hipGetLastError();
}

hipError_t launch_iota(uint32_t *v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3((unsigned)blocks_for(n, 256)), dim3(256), 0, st, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks_for(n, 256)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

uint64_t emit_blocks(uint64_t capacity) { return (capacity + kEmitSpan - 1) / kEmitSpan; }

hipError_t launch_emit(const uint32_t *order, const uint32_t *n_tiles, const uint2 *rect, const uint32_t *offs,
                       int64_t n, uint32_t *part, const uint32_t *m_dev, const EmitFrames &frames,
                       uint64_t capacity, uint32_t *inst_tile, uint32_t *inst_gauss, int32_t *overflow,
                       hipStream_t st) {
    if (n <= 0 || capacity == 0) return hipSuccess;
    const uint64_t nb = emit_blocks(capacity);
    hipLaunchKernelGGL(k_emit_partition, dim3((unsigned)blocks_for(n, kThreads)), dim3(kThreads), 0, st, order,
                       n_tiles, offs, n, nb, part);
    hipLaunchKernelGGL(k_emit, dim3((unsigned)nb), dim3(kThreads), 0, st, order, n_tiles, rect, offs, n,
                       (const uint32_t *)part, m_dev, frames, capacity, inst_tile, inst_gauss, overflow);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t *inst_tile, const uint32_t *m_dev, uint64_t capacity, uint2 *ranges,
                              uint32_t n_tiles_total, hipStream_t st) {
    if (capacity == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)blocks_for((int64_t)capacity, kThreads)), dim3(kThreads), 0,
                       st, inst_tile, m_dev, capacity, ranges, n_tiles_total);
    return hipGetLastError();
}

}  // namespace omnigs
