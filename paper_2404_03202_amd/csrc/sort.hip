// sort.hip -- binning of Gaussian instances into 16x16 tiles (Sec. 3.3: one
// instance per Gaussian and tile its footprint covers), ordered by the
// distance t_r inside each tile (Sec. 3.3: the ERP model orders by t_r, not
// t_z).
//
// Instead of one wide (tile | depth) key sort over all M instances, the
// order is built from two narrow stable sorts:
//   1. the N Gaussians are sorted by the float bits of t_r (4 passes over N);
//   2. one entry per (Gaussian, touched block of 8x8 tiles) is emitted in
//      that depth order (a scan of the block counts in depth order gives
//      each Gaussian its output range; every emit workgroup writes a fixed
//      span of consecutive outputs), then the S entries are stably
//      radix-sorted on the block id alone (ceil(log2 blocks / 8) passes);
//      bin.hip expands each block's list into the lists of its tiles.
// The result is each tile's list in (t_r, Gaussian id) order, identical to a
// sort on (tile, t_r, id), at a fraction of the traffic of a 64-bit key sort
// over M.
//
// The LSD radix sort uses 8-bit digits and one kernel per pass after a
// single histogram kernel (the one-sweep scheme of Adinets and Merrill,
// 2022): the histogram kernel counts every pass's digits over the whole
// input at once; in a pass, each block ranks its keys with ballot-based
// matches (8 ballots per key, wave64), publishes its per-digit counts, takes
// the counts of all earlier blocks from their published words (decoupled
// lookback), places its keys in LDS in digit order and writes them out as
// contiguous per-digit runs.  A sort is a clear of its counters (or the
// caller's shared clear), the histogram and the passes: no scan kernels
// between passes.  The exclusive scan below uses the same lookback.
#include "internal.h"

#include <algorithm>

namespace omnigs {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kRadixBits = 8;
constexpr int kBins = 1 << kRadixBits;
constexpr int kScanItems = 16;
constexpr int kScanTile = kThreads * kScanItems;
constexpr int kScanThreads = 512;  // threads of a lookback scan block (kScanTile / 512 items each)
constexpr int kEmitItems = 8;
constexpr int kEmitSpan = kThreads * kEmitItems;  // outputs per emit block
static_assert(kEmitItems == 8, "k_emit stores a thread's outputs as two uint4");

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

// The same over the NT threads of a block (NT / 64 waves).
template <int NT>
__device__ inline uint32_t block_exclusive_scan_n(uint32_t v, uint32_t *wave_tot, uint32_t *total) {
    constexpr int NW = NT / kWave;
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
    for (int k = 0; k < NW; ++k) {
        const uint32_t t = wave_tot[k];
        base += (k < w) ? t : 0u;
        all += t;
    }
    if (threadIdx.x == 0) *total = all;
    __syncthreads();
    return base + x - v;
}

// A pass runs 512 threads (eight waves, kPI keys each) per block: more waves
// per compute unit hide more of the ranking's and the loads' latency; the
// first kBins threads own a digit each.  Blocks hold 4096 keys, or 6144 once
// that still gives every compute unit a block (fewer blocks, shorter
// lookback chains).
constexpr int kPassThreads = 512;
constexpr int kPassWaves = kPassThreads / kWave;
constexpr int kSmallItems = 8, kLargeItems = 12;
static_assert(kPassThreads >= kBins, "pass layout");
constexpr int64_t kLargeFrom = (int64_t)256 * kPassThreads * kLargeItems;

// Keys per block of a sort of n keys.
int64_t pass_tile_keys(int64_t n) { return (int64_t)kPassThreads * (n >= kLargeFrom ? kLargeItems : kSmallItems); }

// ---------------------------------------------------------------- radix pass
// Element count of a sort: n, or min(n, *n_dev) when counted on the device.
__device__ inline int64_t sort_count(int64_t n, const uint32_t *n_dev) {
    if (!n_dev) return n;
    const int64_t m = *n_dev;
    return m < n ? m : n;
}

// Lookback words: 0 until published, then count + 1 of one digit, the top
// bit set when the count is inclusive (this block and all earlier ones)
// rather than this block's own.  Counts stay below 2^31 - 1 (checked on the
// host).
constexpr uint32_t kInc = 1u << 31, kCountMask = kInc - 1u;
constexpr int kMaxPasses = 4;
constexpr int kHeadWords = kMaxPasses * kBins + 64;  // digit totals, then one ticket per pass
// Bound on the polls of one lookback word: an earlier block always publishes
// (blocks take their position from a ticket, so every earlier position is
// held by a block that is already running), the bound only guarantees that
// the kernel ends whatever happens.  A wait that reaches it sets bit 0 of
// the call's fault word (when given): the prefix it continues with is then
// wrong, and the caller is told so.
constexpr uint32_t kMaxPolls = 1u << 20;
uint32_t g_max_polls = kMaxPolls;  // lowered only by the lookback self-test
#ifndef OMNIGS_SORT_LOOK
#define OMNIGS_SORT_LOOK 4
#endif
constexpr int kLook = OMNIGS_SORT_LOOK;  // lookback words loaded at once

// Digit totals of every pass over the whole input (one read of the keys);
// ghist is zero on entry.  Each block takes chunks of kHistChunk keys (all
// loads of a chunk issued before its counts), counts them in per-wave LDS
// histograms and adds its nonzero totals to ghist once.
constexpr int kHistThreads = 512;  // eight waves: more loads in flight per compute unit
constexpr int kHistWaves = kHistThreads / kWave;
constexpr int kHistItems = 8;
constexpr int kHistChunk = kHistThreads * kHistItems;
constexpr int kHistMaxBlocks = 256;  // bounds the global atomics per digit
__global__ __launch_bounds__(kHistThreads) void k_sort_hist(const uint32_t *keys, int64_t n_max,
                                                             const uint32_t *n_dev, int passes, int bits,
                                                             uint32_t *ghist) {
    __shared__ uint32_t h[kHistWaves][kMaxPasses * kBins];
    for (int k = threadIdx.x; k < kHistWaves * kMaxPasses * kBins; k += kHistThreads) (&h[0][0])[k] = 0;
    __syncthreads();
    const int64_t n = sort_count(n_max, n_dev);
    const int w = threadIdx.x / kWave;
    for (int64_t c0 = (int64_t)blockIdx.x * kHistChunk; c0 < n; c0 += (int64_t)gridDim.x * kHistChunk) {
        uint32_t key[kHistItems];
#pragma unroll
        for (int it = 0; it < kHistItems; ++it) {
            const int64_t idx = c0 + it * kHistThreads + threadIdx.x;
            key[it] = idx < n ? keys[idx] : 0u;
        }
#pragma unroll
        for (int it = 0; it < kHistItems; ++it) {
            if (c0 + it * kHistThreads + threadIdx.x >= n) continue;
            for (int p = 0; p < passes; ++p) {
                const int pb = min(kRadixBits, bits - p * kRadixBits);
                atomicAdd(&h[w][p * kBins + ((key[it] >> (p * kRadixBits)) & ((1u << pb) - 1u))], 1u);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < passes * kBins; k += kHistThreads) {
        uint32_t t = 0;
#pragma unroll
        for (int q = 0; q < kHistWaves; ++q) t += h[q][k];
        if (t) atomicAdd(&ghist[k], t);
    }
}

// One pass: the block at ticket position b ranks its kTK keys by digit
// (ballot matches per wave), publishes its digit counts, looks back over the
// earlier blocks' words for the count of each digit before it (decoupled
// lookback), and writes its keys as contiguous per-digit runs at
// (keys of smaller digits) + (earlier blocks' keys of the same digit) +
// (rank in the block).  vals_in == nullptr: the values are the input
// positions.  key_ranges (one-pass sorts, may be null): workgroup 0 writes
// [start, end) of every key value below n_ranges from the digit totals.
template <int kPI>
__global__ __launch_bounds__(kPassThreads) void k_radix_pass(const uint32_t *keys_in, const uint32_t *vals_in,
                                                          uint32_t *keys_out, uint32_t *vals_out, int64_t n_max,
                                                          const uint32_t *n_dev, int shift, int bits,
                                                          const uint32_t *ghist, uint32_t *status,
                                                          uint32_t *ticket, uint2 *key_ranges, int n_ranges,
                                                          uint32_t *fault, uint32_t max_polls) {
    constexpr int kTK = kPassThreads * kPI;  // keys per block
    __shared__ uint32_t s_keys[kTK];
    __shared__ uint32_t s_vals[kTK];
    __shared__ uint32_t cnt[kPassWaves][kBins];
    __shared__ uint32_t gbase[kBins];
    __shared__ uint32_t wave_tot[kPassWaves];
    __shared__ uint32_t total;
    __shared__ uint32_t s_pos;
    const int64_t n = sort_count(n_max, n_dev);
    if (key_ranges && blockIdx.x == 0) {
        const uint32_t c = threadIdx.x < kBins ? ghist[threadIdx.x] : 0u;
        const uint32_t start = block_exclusive_scan_n<kPassThreads>(c, wave_tot, &total);
        if ((int)threadIdx.x < n_ranges) key_ranges[threadIdx.x] = make_uint2(start, start + c);
    }
    // the first ceil(n / kTK) workgroups take the tickets 0, 1, ... in
    // the order they start; the others (a grid sized for a capacity) have no
    // keys and leave at once
    if ((int64_t)blockIdx.x * kTK >= n) return;
    if (threadIdx.x == 0) s_pos = atomicAdd(ticket, 1u);
    // keys of digit threadIdx.x (0 past the pass's digits)
    const uint32_t gcount = threadIdx.x < kBins ? ghist[threadIdx.x] : 0u;
    for (int k = threadIdx.x; k < kPassWaves * kBins; k += kPassThreads) (&cnt[0][0])[k] = 0;
    __syncthreads();
    const uint32_t b = s_pos;
    const int64_t block0 = (int64_t)b * kTK;
    const int w = threadIdx.x / kWave, lane = __lane_id();
    const uint32_t mask = (1u << bits) - 1u;
    const int64_t base = block0 + (int64_t)w * (kPI * kWave);
    uint32_t key[kPI], val[kPI], rank[kPI];
    // keys past n get the largest digit: they sort last in the block and are
    // never written out
#pragma unroll
    for (int it = 0; it < kPI; ++it) {
        const int64_t idx = base + it * kWave + lane;
        const bool valid = idx < n;
        key[it] = valid ? keys_in[idx] : 0xffffffffu;
        val[it] = valid ? (vals_in ? vals_in[idx] : (uint32_t)idx) : 0u;
    }
#pragma unroll
    for (int it = 0; it < kPI; ++it) {
        const int64_t idx = base + it * kWave + lane;
        const uint32_t d = (idx < n) ? (key[it] >> shift) & mask : mask;
        const uint64_t peers = match_digit(d, bits, true);
        const uint32_t before = cnt[w][d];
        rank[it] = before + (uint32_t)__popcll(peers & lanemask_lt());
        if ((peers & lanemask_lt()) == 0) cnt[w][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    const int d = threadIdx.x;  // the digit of the first kBins threads
    uint32_t per[kPassWaves], tot = 0;
#pragma unroll
    for (int k = 0; k < kPassWaves; ++k) {
        per[k] = d < kBins ? cnt[k][d] : 0u;
        tot += per[k];
    }
    // padding keys (digit `mask`) are not counted
    const int64_t nvalid64 = n - block0 < kTK ? n - block0 : kTK;
    const uint32_t pad = (uint32_t)(kTK - nvalid64);
    const uint32_t mine = d == (int)mask ? tot - pad : tot;
    uint32_t before = 0;  // keys of digit d in the earlier blocks
    if (d <= (int)mask) {
        uint32_t *word = status + (int64_t)b * kBins + d;
        __hip_atomic_store(word, (b == 0 ? kInc : 0u) | (mine + 1u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (b > 0) {
            // windows of kLook earlier blocks, loaded together: sum their own
            // counts back to the first inclusive word; an unpublished word is
            // polled again from its position
            int64_t p = (int64_t)b - 1;
            uint32_t polls = 0;
            for (;;) {
                uint32_t v[kLook];
#pragma unroll
                for (int i = 0; i < kLook; ++i)
                    v[i] = p - i >= 0 ? __hip_atomic_load(status + (p - i) * kBins + d, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT)
                                      : kInc | 1u;  // before block 0: nothing
                int used = 0;
                bool inc = false, wait = false;
#pragma unroll
                for (int i = 0; i < kLook; ++i) {
                    if (inc || wait) continue;
                    if (v[i] == 0u) {
                        wait = true;
                        continue;
                    }
                    before += (v[i] & kCountMask) - 1u;
                    inc = (v[i] & kInc) != 0u;
                    ++used;
                }
                if (inc) break;
                p -= used;
                if (wait) {
                    if (++polls >= max_polls) {
                        if (fault) atomicOr(fault, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __hip_atomic_store(word, kInc | (before + mine + 1u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    // block layout: digit runs in order, each wave's keys after the earlier
    // waves' keys of the same digit
    const uint32_t start = block_exclusive_scan_n<kPassThreads>(tot, wave_tot, &total);
    if (d < kBins) {
        uint32_t run = start;
#pragma unroll
        for (int k = 0; k < kPassWaves; ++k) {
            cnt[k][d] = run;
            run += per[k];
        }
    }
    // first output position of digit d: the keys of all smaller digits
    const uint32_t gstart = block_exclusive_scan_n<kPassThreads>(gcount, wave_tot, &total);
    if (d <= (int)mask) gbase[d] = gstart + before - start;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kPI; ++it) {
        const int64_t idx = base + it * kWave + lane;
        const uint32_t dg = (idx < n) ? (key[it] >> shift) & mask : mask;
        const uint32_t pos = cnt[w][dg] + rank[it];
        s_keys[pos] = key[it];
        s_vals[pos] = val[it];
    }
    __syncthreads();
    const int nvalid = (int)nvalid64;
    for (int q = threadIdx.x; q < nvalid; q += kPassThreads) {
        const uint32_t k = s_keys[q];
        const uint32_t dg = (k >> shift) & mask;
        const uint32_t dst = gbase[dg] + (uint32_t)q;
        if (dst < (uint64_t)n) {
            keys_out[dst] = k;
            vals_out[dst] = s_vals[q];
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

// Item idx of a scan with exclusive value o and count c: the emit blocks
// whose first output lies in [o, o + c) start in rank idx.
__device__ inline void mark_partition(const ScanPartition &P, int64_t idx, uint32_t o, uint32_t c) {
    if (c == 0) return;
    const uint64_t b1 = ((uint64_t)o + c - 1) / kEmitSpan;
    for (uint64_t b = ((uint64_t)o + kEmitSpan - 1) / kEmitSpan; b <= b1 && b < P.blocks; ++b) P.part[b] = (uint32_t)idx;
}

// Single-pass exclusive scan of kScanTile-element tiles: the workgroup at
// ticket position b loads its tile (all loads issued before use), publishes
// the tile sum, and its first wave takes the sum of all earlier tiles by
// decoupled lookback over 64 earlier status words per round (the nearest
// inclusive word ends it); the tile is then scanned with that offset.
// status: one 64-bit word per tile, zero until published, then value + 1
// with the top bit set when the value is inclusive.
constexpr uint64_t kInc64 = 1ull << 63;
__global__ __launch_bounds__(kScanThreads) void k_scan_lookback(const uint32_t *in, const uint32_t *gather, uint32_t *out,
                                                             int64_t n, uint64_t *status, uint32_t *ticket,
                                                             uint32_t *grand_total, uint32_t *fault,
                                                             uint32_t max_polls, ScanPartition P) {
    constexpr int kSI = kScanTile / kScanThreads;  // items per thread
    __shared__ uint32_t wave_tot[kScanThreads / kWave];
    __shared__ uint32_t total;
    __shared__ uint32_t s_data[kScanTile];
    __shared__ uint32_t s_pos;
    __shared__ uint64_t s_before;
    if (threadIdx.x == 0) s_pos = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t b = s_pos;
    const int64_t block0 = (int64_t)b * kScanTile;
    uint32_t v[kSI];
#pragma unroll
    for (int it = 0; it < kSI; ++it) {
        const int64_t idx = block0 + it * kScanThreads + threadIdx.x;
        v[it] = idx < n ? scan_input(in, gather, idx, n) : 0u;
    }
#pragma unroll
    for (int it = 0; it < kSI; ++it) s_data[it * kScanThreads + threadIdx.x] = v[it];
    __syncthreads();
    // blocked arrangement: thread t owns items [t*kSI, (t+1)*kSI)
    uint32_t s = 0;
#pragma unroll
    for (int it = 0; it < kSI; ++it) {
        v[it] = s_data[threadIdx.x * kSI + it];
        s += v[it];
    }
    uint32_t run = block_exclusive_scan_n<kScanThreads>(s, wave_tot, &total);
    if (threadIdx.x < kWave) {
        const int lane = __lane_id();
        const uint64_t agg = total;
        if (lane == 0)
            __hip_atomic_store(status + b, (b == 0 ? kInc64 : 0ull) | (agg + 1ull), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        uint64_t before = 0;
        int64_t p = (int64_t)b - 1;  // nearest earlier tile not yet summed
        uint32_t polls = 0;
        while (p >= 0) {
            const int64_t q = p - lane;
            const uint64_t w = q >= 0 ? __hip_atomic_load(status + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                      : kInc64 | 1ull;  // before tile 0: nothing
            const uint64_t incs = __ballot((w & kInc64) != 0ull);
            const int first_inc = incs ? __builtin_ctzll(incs) : kWave;
            const uint64_t need = first_inc < kWave ? (2ull << first_inc) - 1ull : ~0ull;  // lanes 0..first_inc
            const uint64_t zeros = __ballot(w == 0ull) & need;
            const int upto = zeros ? __builtin_ctzll(zeros) : (first_inc < kWave ? first_inc + 1 : kWave);
            uint64_t c = lane < upto ? (w & ~kInc64) - 1ull : 0ull;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) c += __shfl_xor(c, off, kWave);
            before += c;
            if (!zeros && first_inc < kWave) break;
            p -= upto;
            if (zeros) {
                if (++polls >= max_polls) {
                    if (fault && lane == 0) atomicOr(fault, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        if (lane == 0) {
            if (b > 0)
                __hip_atomic_store(status + b, kInc64 | (before + agg + 1ull), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            s_before = before;
        }
    }
    __syncthreads();
    run += (uint32_t)s_before;
#pragma unroll
    for (int it = 0; it < kSI; ++it) {
        s_data[threadIdx.x * kSI + it] = run;
        if (P.part) mark_partition(P, block0 + threadIdx.x * kSI + it, run, v[it]);
        run += v[it];
    }
    if (grand_total && block0 + kScanTile >= n && threadIdx.x == kScanThreads - 1) *grand_total = run;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSI; ++it) {
        const int64_t idx = block0 + it * kScanThreads + threadIdx.x;
        if (idx < n) out[idx] = s_data[it * kScanThreads + threadIdx.x];
    }
}

// Exclusive scan of at most kScanTile elements in one workgroup (blocked
// arrangement: thread t owns items [t*kScanItems, (t+1)*kScanItems)).
__global__ __launch_bounds__(kThreads) void k_scan_tile(const uint32_t *in, const uint32_t *gather, uint32_t *out,
                                                         int64_t n, uint32_t *grand_total, ScanPartition P) {
    __shared__ uint32_t wave_tot[kWaves];
    __shared__ uint32_t total;
    __shared__ uint32_t s_data[kScanTile];
    uint32_t v[kScanItems];
#pragma unroll
    for (int it = 0; it < kScanItems; ++it) {
        const int64_t idx = it * kThreads + threadIdx.x;
        v[it] = idx < n ? scan_input(in, gather, idx, n) : 0u;
    }
#pragma unroll
    for (int it = 0; it < kScanItems; ++it) s_data[it * kThreads + threadIdx.x] = v[it];
    __syncthreads();
    uint32_t s = 0;
#pragma unroll
    for (int it = 0; it < kScanItems; ++it) {
        v[it] = s_data[threadIdx.x * kScanItems + it];
        s += v[it];
    }
    uint32_t run = block_exclusive_scan(s, wave_tot, &total);
#pragma unroll
    for (int it = 0; it < kScanItems; ++it) {
        s_data[threadIdx.x * kScanItems + it] = run;
        if (P.part) mark_partition(P, threadIdx.x * kScanItems + it, run, v[it]);
        run += v[it];
    }
    if (grand_total && threadIdx.x == kThreads - 1) *grand_total = run;
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kScanItems; ++it) {
        const int64_t idx = it * kThreads + threadIdx.x;
        if (idx < n) out[idx] = s_data[it * kThreads + threadIdx.x];
    }
}

// ---------------------------------------------------------------- emission
// Entries are emitted in depth order: rank r of the depth order owns the
// output range [offs[r], offs[r] + count(r)), count = tiles or super-tiles of
// its rectangle (the scan behind offs used the same count).  Every emit block writes a
// fixed span of kEmitSpan consecutive outputs, whatever the tile counts of the
// Gaussians behind them (the nearest Gaussians, which come first, cover up to
// thousands of tiles each).  part[b] = the rank owning output b * kEmitSpan.
__global__ __launch_bounds__(kThreads) void k_emit_partition(const uint32_t *offs, const uint32_t *m_dev, int64_t n,
                                                              uint64_t part_blocks, uint32_t *part) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= n) return;
    // rank r's count from the adjacent offsets (the last rank ends at M)
    const uint64_t o = offs[r];
    const uint64_t e = r + 1 < n ? (uint64_t)offs[r + 1] : (uint64_t)*m_dev;
    if (e <= o) return;
    const uint64_t b1 = (e - 1) / kEmitSpan;
    for (uint64_t b = (o + kEmitSpan - 1) / kEmitSpan; b <= b1 && b < part_blocks; ++b) part[b] = (uint32_t)r;
}

__global__ __launch_bounds__(kThreads) void k_emit(const uint32_t *order, const uint2 *rect,
                                                    const uint32_t *offs, int64_t n, const uint32_t *part,
                                                    const uint32_t *m_dev, EmitFrames F, uint64_t capacity,
                                                    uint32_t *inst_tile, uint32_t *inst_gauss, int32_t *overflow) {
    __shared__ uint32_t s_off[kEmitSpan + 1];
    __shared__ uint32_t s_gid[kEmitSpan + 1];
    __shared__ uint2 s_rect[kEmitSpan + 1];  // the tile rectangle
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
    // the ranks' records, in two rounds of loads (ids and offsets, then the
    // gathered rectangles) each issued whole before use; a culled record's
    // rectangle is empty, so no count is gathered
    constexpr int kRankIters = (kEmitSpan + kThreads) / kThreads;  // covers kEmitSpan + 1 ranks
    uint32_t gv[kRankIters], ov[kRankIters];
    uint2 rv[kRankIters];
#pragma unroll
    for (int it = 0; it < kRankIters; ++it) {
        const int i = threadIdx.x + it * kThreads;
        gv[it] = i < cnt ? order[r0 + i] : 0xffffffffu;
        ov[it] = i < cnt ? offs[r0 + i] : 0u;
    }
#pragma unroll
    for (int it = 0; it < kRankIters; ++it) rv[it] = gv[it] < (uint64_t)n ? rect[gv[it]] : make_uint2(0, 0);
#pragma unroll
    for (int it = 0; it < kRankIters; ++it) {
        const int i = threadIdx.x + it * kThreads;
        if (i >= cnt) continue;
        const uint32_t g = gv[it];
        // camera of record g = b * n_per + i
        const int cam = F.count > 1 && g < (uint64_t)n ? (int)min((int64_t)g / F.n_per, (int64_t)F.count - 1) : 0;
        s_off[i] = ov[it];
        s_gid[i] = g;
        s_rect[i] = rv[it];
        s_cam[i] = (uint8_t)cam;
    }
    __syncthreads();
    uint64_t jend = j0 + kEmitSpan;
    if (jend > M) jend = M;
    if (jend > capacity) jend = capacity;
    // thread t writes the kEmitItems consecutive outputs from j0 + t kEmitItems:
    // one search for the rank owning the first (the last rank i with
    // s_off[i] <= j), then the owner only moves forward
    const uint64_t jt = j0 + (uint64_t)threadIdx.x * kEmitItems;
    if (jt >= jend) return;
    int lo = 0;
    {
        int hi = cnt;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (s_off[mid] <= jt) lo = mid; else hi = mid;
        }
    }
    uint32_t tile[kEmitItems], gid[kEmitItems];
    // the owner's rectangle (in super-tiles when emitting super entries),
    // formed again only when the owner changes
    int cur = -1, cam = 0;
    uint2 tr = make_uint2(0u, 0u), rc = tr;
#pragma unroll
    for (int i = 0; i < kEmitItems; ++i) {
        const uint64_t j = jt + i;
        tile[i] = gid[i] = 0u;
        if (j >= jend) continue;
        while (lo + 1 < cnt && s_off[lo + 1] <= j) ++lo;
        if (lo != cur) {
            cur = lo;
            tr = s_rect[lo];
            cam = s_cam[lo];
            rc = F.super ? super_rect(tr, F.tiles_x[cam]) : tr;
        }
        const uint32_t k = (uint32_t)(j - s_off[lo]);
        const uint32_t ntx = rc.x >> 16, tx0 = rc.x & 0xffffu, ty0 = rc.y & 0xffffu;
        if (ntx == 0) continue;
        const uint32_t cols = (uint32_t)F.cols[cam];
        const uint32_t ty = ty0 + k / ntx;
        uint32_t tx = tx0 + k % ntx;
        if (tx >= cols) tx -= cols;
        tile[i] = F.base[cam] + ty * cols + tx;
        if (F.super && F.cover_key) tile[i] |= cover_bits(cover_of(tr, F.tiles_x[cam], (int)tx, (int)ty));
        gid[i] = s_gid[lo];
    }
    if (jt + kEmitItems <= jend) {
        // whole run: two 16-byte stores per array (jt is a multiple of 8)
        uint4 *dt = reinterpret_cast<uint4 *>(inst_tile + jt), *dg = reinterpret_cast<uint4 *>(inst_gauss + jt);
        dt[0] = make_uint4(tile[0], tile[1], tile[2], tile[3]);
        dt[1] = make_uint4(tile[4], tile[5], tile[6], tile[7]);
        dg[0] = make_uint4(gid[0], gid[1], gid[2], gid[3]);
        dg[1] = make_uint4(gid[4], gid[5], gid[6], gid[7]);
    } else {
#pragma unroll
        for (int i = 0; i < kEmitItems; ++i)
            if (jt + i < jend) {
                inst_tile[jt + i] = tile[i];
                inst_gauss[jt + i] = gid[i];
            }
    }
}

// [start, end) of every tile from adjacent sorted instances.  Ranges must be
// zeroed beforehand (empty tiles keep [0, 0)).
__global__ __launch_bounds__(kThreads) void k_tile_ranges(const uint32_t *inst_tile, const uint32_t *m_dev,
                                                           uint64_t capacity, uint2 *ranges, uint32_t n_tiles_total,
                                                           uint32_t key_mask) {
    const uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    uint64_t m = *m_dev;
    if (m > capacity) m = capacity;
    if (i >= m) return;
    const uint32_t t = inst_tile[i] & key_mask;
    if (t >= n_tiles_total) return;
    if (i == 0 || (inst_tile[i - 1] & key_mask) != t) ranges[t].x = (uint32_t)i;
    if (i + 1 == m || (inst_tile[i + 1] & key_mask) != t) ranges[t].y = (uint32_t)(i + 1);
}

// Region blockIdx.y of the list, grid-strided in x.
// Sets words [i, i + 4) of p[0, n) to v: one 16-byte store when they lie
// inside and p + i is 16-byte aligned, else word by word.
__device__ inline void fill4(uint32_t *p, int64_t n, int64_t i, uint32_t v) {
    if (i + 4 <= n && ((reinterpret_cast<uintptr_t>(p + i) & 15u) == 0)) {
        *reinterpret_cast<uint4 *>(p + i) = make_uint4(v, v, v, v);
    } else {
        for (int64_t k = i; k < i + 4 && k < n; ++k) p[k] = v;
    }
}

__global__ __launch_bounds__(256) void k_clear_list(ClearList L) {
    const int r = blockIdx.y;
    uint32_t *p = L.p[r];
    const int64_t n = L.n[r];
    for (int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4; i < n; i += (int64_t)gridDim.x * 1024)
        fill4(p, n, i, 0u);
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i < n) fill4(p, n, i, v);
}

int64_t blocks_for(int64_t n, int64_t per) { return (n + per - 1) / per; }

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
    // one status word per tile, then the ticket
    return ((size_t)blocks_for(n > 0 ? n : 1, kScanTile) * 8 + 64 + 255) / 256 * 256 + 256;
}

int64_t scan_clear_words(int64_t n) {
    const int64_t nb = blocks_for(n > 0 ? n : 1, kScanTile);
    return nb == 1 ? 0 : nb * 2 + 1;  // the status words and the ticket, as u32
}

hipError_t scan_exclusive(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total, void *scratch,
                          hipStream_t st, const uint32_t *gather, bool cleared, uint32_t *fault, ScanPartition P) {
    if (n <= 0) return total ? launch_fill_u32(total, 0u, 1, st) : hipSuccess;
    const int64_t nb = blocks_for(n, kScanTile);
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_tile, dim3(1), dim3(kThreads), 0, st, in, gather, out, n, total, P);
        return hipGetLastError();
    }
    uint64_t *status = static_cast<uint64_t *>(scratch);
    uint32_t *ticket = reinterpret_cast<uint32_t *>(status + nb);
    const int64_t words = scan_clear_words(n);
    if (!cleared) {
        const hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t *>(status), 0u, words, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_scan_lookback, dim3((unsigned)nb), dim3(kScanThreads), 0, st, in, gather, out, n, status, ticket,
                       total, fault, g_max_polls, P);
    return hipGetLastError();
}

size_t sort_scratch_bytes(int64_t n) {
    const int64_t nb = blocks_for(n > 0 ? n : 1, pass_tile_keys(n));
    return ((size_t)kHeadWords + (size_t)kMaxPasses * nb * kBins) * 4 + 256;
}

int64_t sort_clear_words(int64_t n, int bits) {
    if (n <= 0) return 0;
    bits = std::min(std::max(bits, 1), 32);
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    return kHeadWords + (int64_t)passes * blocks_for(n, pass_tile_keys(n)) * kBins;
}

hipError_t radix_sort_pairs(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_tmp,
                            uint32_t *vals_tmp, uint32_t *keys_out, uint32_t *vals_out, int64_t n, int bits,
                            void *scratch, hipStream_t st, const uint32_t *n_dev, uint2 *key_ranges,
                            int n_ranges, bool cleared, uint32_t *fault) {
    if (key_ranges && (bits > kRadixBits || n_ranges > kBins)) return hipErrorInvalidValue;
    if (n <= 0)
        return key_ranges && n_ranges > 0
                   ? launch_fill_u32(reinterpret_cast<uint32_t *>(key_ranges), 0u, (int64_t)2 * n_ranges, st)
                   : hipSuccess;
    if (n >= (int64_t)kCountMask) return hipErrorInvalidValue;  // lookback words hold count + 1 in 31 bits
    if (bits < 1) bits = 1;
    if (bits > 32) bits = 32;
    const int passes = (bits + kRadixBits - 1) / kRadixBits;
    const int64_t nb = blocks_for(n, pass_tile_keys(n));
    const bool large = n >= kLargeFrom;
    // [digit totals per pass | tickets | lookback words per pass], cleared at once
    uint32_t *head = static_cast<uint32_t *>(scratch);
    uint32_t *ghist = head, *tickets = head + kMaxPasses * kBins;
    uint32_t *status = head + kHeadWords;
    const int64_t words = sort_clear_words(n, bits);
    if (!cleared) {
        const hipError_t e = launch_fill_u32(head, 0u, words, st);
        if (e != hipSuccess) return e;
    }
    const int64_t hist_blocks = std::min<int64_t>(blocks_for(n, kHistChunk), kHistMaxBlocks);
    hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)hist_blocks), dim3(kHistThreads), 0, st, keys_in, n, n_dev, passes,
                       bits, ghist);
    // ping-pong so that the last pass lands in keys_out / vals_out
    const uint32_t *src_k = keys_in, *src_v = vals_in;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * kRadixBits;
        const int pbits = std::min(kRadixBits, bits - shift);
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        uint32_t *dk = to_out ? keys_out : keys_tmp;
        uint32_t *dv = to_out ? vals_out : vals_tmp;
        const uint32_t *gh = ghist + p * kBins;
        uint32_t *stp = status + (int64_t)p * nb * kBins;
        if (large)
            hipLaunchKernelGGL(k_radix_pass<kLargeItems>, dim3((unsigned)nb), dim3(kPassThreads), 0, st, src_k, src_v,
                               dk, dv, n, n_dev, shift, pbits, gh, stp, tickets + p, key_ranges, n_ranges, fault,
                               g_max_polls);
        else
            hipLaunchKernelGGL(k_radix_pass<kSmallItems>, dim3((unsigned)nb), dim3(kPassThreads), 0, st, src_k, src_v,
                               dk, dv, n, n_dev, shift, pbits, gh, stp, tickets + p, key_ranges, n_ranges, fault,
                               g_max_polls);
        src_k = dk;
        src_v = dv;
    }
    return hipGetLastError();
}

hipError_t launch_clear(const ClearList &L, hipStream_t st) {
    if (L.count == 0) return hipSuccess;
    int64_t most = 0;
    for (int k = 0; k < L.count; ++k) most = std::max(most, L.n[k]);
    const unsigned bx = (unsigned)std::min<int64_t>(blocks_for(most, 1024), 2048);
    hipLaunchKernelGGL(k_clear_list, dim3(bx, (unsigned)L.count), dim3(256), 0, st, L);
    return hipGetLastError();
}

void set_lookback_poll_limit(uint32_t polls) { g_max_polls = polls ? polls : kMaxPolls; }

namespace {
__global__ void k_selftest_keys(uint32_t *keys, int64_t n, uint32_t mask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) keys[i] = selftest_key((uint32_t)i) & mask;
}
}  // namespace

hipError_t launch_selftest_keys(uint32_t *keys, int64_t n, uint32_t mask, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_selftest_keys, dim3((unsigned)blocks_for(n, 256)), dim3(256), 0, st, keys, n, mask);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks_for(n, 1024)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

uint64_t emit_blocks(uint64_t capacity) { return (capacity + kEmitSpan - 1) / kEmitSpan; }

hipError_t launch_emit(const uint32_t *order, const uint2 *rect, const uint32_t *offs, int64_t n, uint32_t *part,
                       const uint32_t *m_dev, const EmitFrames &frames, uint64_t capacity, uint32_t *inst_tile,
                       uint32_t *inst_gauss, int32_t *overflow, hipStream_t st, bool partitioned) {
    if (n <= 0 || capacity == 0) return hipSuccess;
    const uint64_t nb = emit_blocks(capacity);
    if (!partitioned)
        hipLaunchKernelGGL(k_emit_partition, dim3((unsigned)blocks_for(n, kThreads)), dim3(kThreads), 0, st, offs,
                           m_dev, n, nb, part);
    hipLaunchKernelGGL(k_emit, dim3((unsigned)nb), dim3(kThreads), 0, st, order, rect, offs, n,
                       (const uint32_t *)part, m_dev, frames, capacity, inst_tile, inst_gauss, overflow);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t *inst_tile, const uint32_t *m_dev, uint64_t capacity, uint2 *ranges,
                              uint32_t n_tiles_total, uint32_t key_mask, hipStream_t st) {
    if (capacity == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)blocks_for((int64_t)capacity, kThreads)), dim3(kThreads), 0,
                       st, inst_tile, m_dev, capacity, ranges, n_tiles_total, key_mask);
    return hipGetLastError();
}

}  // namespace omnigs
