// Stable LSD radix sort of (u32 key, u32 value) pairs for gfx950 (the
// RadixSortPairs step of Algorithm 1), and the per-pixel segment ranges of
// the sorted fragment list.
//
// Each pass over a digit of D bits is reduce-then-scan:
//   upsweep   one LDS histogram per tile (wave-level digit matching, so a
//             digit shared by many lanes costs one LDS update per wave);
//   scan      per-digit exclusive scan over tiles, then over digits;
//   downsweep the tile is ranked stably inside LDS (per-wave multisplit,
//             cross-wave prefix per digit), staged in LDS in digit order and
//             written out so that consecutive lanes write consecutive
//             addresses of one digit's run.
// The live element count may sit in device memory (fragment count M), so a
// pass needs no host round trip; blocks past the live count exit at once.
#include "internal.h"

namespace inpc {

constexpr int kSortBlock = 512;   // 8 waves per sort tile
constexpr uint32_t kXcdGroup = 8;   // consecutive downsweep tiles per XCD

static inline size_t tiles_for(int items, int64_t n) {
    const int64_t tile = (int64_t)kSortBlock * items;
    return (size_t)((n + tile - 1) / tile);
}

size_t sort_counts_words(int digit, int items, int64_t n_bound) {
    return ((size_t)1 << digit) * (tiles_for(items, n_bound) + 1) + ((size_t)1 << digit);
}

int radix_passes(int digit, int bits) { return bits <= 0 ? 0 : (bits + digit - 1) / digit; }

__device__ __forceinline__ uint32_t live_count(const uint32_t* n_dev, uint32_t n_bound) {
    if (!n_dev) return n_bound;
    const uint32_t n = *n_dev;
    return n < n_bound ? n : n_bound;
}

// DROP: keys equal to drop_key are left out (counted nowhere, written nowhere).
template <int D, int ITEMS, bool DROP>
__global__ __launch_bounds__(kSortBlock) void k_radix_upsweep(const uint32_t* __restrict__ keys,
                                                              const uint32_t* __restrict__ n_dev,
                                                              uint32_t n_bound, int shift,
                                                              uint32_t* __restrict__ counts,
                                                              uint32_t stride, uint32_t drop_key) {
    // One LDS histogram per wave.  A row whose lanes all carry the same digit
    // (common once the lower digits are sorted) costs a single update; other
    // rows use per-lane LDS atomics.
    constexpr int BINS = 1 << D;
    constexpr int TILE = kSortBlock * ITEMS;
    constexpr int WAVES = kSortBlock / kWave;
    __shared__ uint32_t s_hist[WAVES][BINS];
    const uint32_t n = live_count(n_dev, n_bound);
    const uint32_t tile = blockIdx.x;
    if ((uint64_t)tile * TILE >= n) return;
    for (int i = threadIdx.x; i < WAVES * BINS; i += kSortBlock) (&s_hist[0][0])[i] = 0;
    __syncthreads();
    const int w = threadIdx.x / kWave, lane = __lane_id();
    const uint32_t base = tile * TILE + w * (ITEMS * kWave);
    uint32_t* h = s_hist[w];
    uint32_t kk[ITEMS];   // every key of the thread in flight before the first is counted
    // Only counts are made, so which lane takes which key does not matter:
    // a wave whose keys all lie below n takes ITEMS consecutive keys per lane
    // with 16-byte loads (ITEMS / 4 loads instead of ITEMS).
    const bool full = base + (uint32_t)(ITEMS * kWave) <= n;
    if (ITEMS % 4 == 0 && full) {
        const uint4* k4 = reinterpret_cast<const uint4*>(keys + base + (uint32_t)lane * ITEMS);
#pragma unroll
        for (int q = 0; q < ITEMS / 4; ++q) {
            const uint4 v = k4[q];
            kk[4 * q] = v.x;
            kk[4 * q + 1] = v.y;
            kk[4 * q + 2] = v.z;
            kk[4 * q + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint32_t idx = base + it * kWave + lane;
            kk[it] = idx < n ? keys[idx] : 0u;
        }
    }
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const uint32_t idx = base + it * kWave + lane;
        const bool valid = (full || idx < n) && !(DROP && kk[it] == drop_key);
        const uint32_t d = valid ? (kk[it] >> shift) & (BINS - 1) : 0u;
        const uint64_t act = __ballot(valid);
        const uint32_t d0 = __shfl(d, 0);
        const uint64_t same = __ballot(valid && d == d0);
        if (same == act && (act & 1ull)) {
            if (lane == 0) h[d0] += (uint32_t)__popcll(act);
        } else if (valid) {
            atomicAdd(&h[d], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < BINS; i += kSortBlock) {
        uint32_t c = 0;
#pragma unroll
        for (int ww = 0; ww < WAVES; ++ww) c += s_hist[ww][i];
        counts[(size_t)i * stride + tile] = c;
    }
}

// Row-wise exclusive scan of counts[bin][0..tiles) in place; bin totals out.
__global__ __launch_bounds__(kSortBlock) void k_scan_rows(uint32_t* __restrict__ counts,
                                                          uint32_t stride,
                                                          const uint32_t* __restrict__ n_dev,
                                                          uint32_t n_bound, uint32_t tile_size,
                                                          uint32_t* __restrict__ totals) {
    __shared__ uint32_t s_tmp[kSortBlock / kWave];
    const uint32_t n = live_count(n_dev, n_bound);
    const uint32_t tiles = (n + tile_size - 1) / tile_size;
    uint32_t* row = counts + (size_t)blockIdx.x * stride;
    uint32_t running = 0;
    for (uint32_t base = 0; base < tiles; base += kSortBlock * 4) {
        const uint32_t i0 = base + threadIdx.x * 4;
        uint32_t v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (i0 + j < tiles) ? row[i0 + j] : 0u;
        const uint32_t s = v[0] + v[1] + v[2] + v[3];
        uint32_t total;
        uint32_t ex = block_excl_sum<kSortBlock>(s, total, s_tmp) + running;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (i0 + j < tiles) row[i0 + j] = ex;
            ex += v[j];
        }
        running += total;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = running;
}

// MODE 0: (key, value) pairs; 1: a second value per key (ain -> aout) moves
// with the pair; 2: as 1, and keys equal to drop_key are left out.
template <int D, int ITEMS, int MODE>
__global__ __launch_bounds__(kSortBlock) void k_radix_downsweep(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, const uint32_t* __restrict__ ain,
    uint32_t* __restrict__ aout, const uint32_t* __restrict__ n_dev,
    uint32_t n_bound, int shift, const uint32_t* __restrict__ row_prefix, uint32_t stride,
    const uint32_t* __restrict__ bin_total, uint32_t drop_key, uint32_t* __restrict__ live_out) {
    constexpr bool DROP = MODE == 2, V2 = MODE >= 1;
    constexpr int BINS = 1 << D;
    constexpr int WAVES = kSortBlock / kWave;
    constexpr int TILE = kSortBlock * ITEMS;
    __shared__ uint32_t s_cnt[WAVES][BINS];   // per-wave digit counts, then cross-wave offsets
    __shared__ uint32_t s_start[BINS];        // first LDS slot of each digit in the tile
    __shared__ uint32_t s_dst[BINS];          // global start of each digit for this tile
    __shared__ uint32_t s_key[TILE];
    __shared__ uint32_t s_val[TILE];
    __shared__ uint32_t s_tmp[WAVES];
    __shared__ uint32_t s_tile_n;             // DROP: items of the tile that take part in the pass

    const uint32_t n = live_count(n_dev, n_bound);
    // Runs of consecutive groups of kXcdGroup tiles go to one XCD (blocks are
    // dealt to the 8 XCDs round-robin): a digit's runs of neighbouring tiles
    // are adjacent in the output, so they meet in one L2 and leave it as
    // whole lines.
    const uint32_t k8 = blockIdx.x >> 3;
    const uint32_t tile = ((k8 / kXcdGroup) * 8u + (blockIdx.x & 7u)) * kXcdGroup + (k8 % kXcdGroup);
    if ((uint64_t)tile * TILE >= n) return;
    for (int i = threadIdx.x; i < WAVES * BINS; i += kSortBlock) (&s_cnt[0][0])[i] = 0;
    __syncthreads();

    const int w = threadIdx.x / kWave, lane = __lane_id();
    const uint32_t base = tile * TILE + w * (ITEMS * kWave);
    uint32_t key[ITEMS], val[ITEMS], rank[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const uint32_t idx = base + it * kWave + lane;
        const bool valid = idx < n;
        key[it] = valid ? kin[idx] : 0u;
        val[it] = valid ? vin[idx] : 0u;
    }
    // Rows are processed in input order, so ranks within a wave are stable.
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const uint32_t idx = base + it * kWave + lane;
        const bool valid = idx < n && !(DROP && key[it] == drop_key);
        const uint32_t d = (key[it] >> shift) & (BINS - 1);
        const uint64_t peers = match_digit<D>(d, valid);
        const uint32_t below = (uint32_t)__popcll(peers & lanemask_lt());
        const int leader = valid ? (__ffsll((unsigned long long)peers) - 1) : lane;
        uint32_t old = 0;
        if (valid && below == 0u) {
            old = s_cnt[w][d];
            s_cnt[w][d] = old + (uint32_t)__popcll(peers);
        }
        old = __shfl(old, leader);
        rank[it] = old + below;
    }
    __syncthreads();
    // Cross-wave exclusive prefix per digit and digit totals of the tile.
    uint32_t my_tot[(BINS + kSortBlock - 1) / kSortBlock];
#pragma unroll
    for (int j = 0; j < (BINS + kSortBlock - 1) / kSortBlock; ++j) {
        const int d = threadIdx.x + j * kSortBlock;
        uint32_t sum = 0;
        if (d < BINS) {
#pragma unroll
            for (int ww = 0; ww < WAVES; ++ww) {
                const uint32_t c = s_cnt[ww][d];
                s_cnt[ww][d] = sum;
                sum += c;
            }
        }
        my_tot[j] = sum;
    }
    // Exclusive scans over digits (digits are owned thread-major: thread t
    // owns digits t, t+256, ...): of this tile's digit totals (LDS slots) and
    // of the global digit totals of the pass (where each digit starts).
    {
        uint32_t running = 0, running_g = 0;   // end: kept items of the tile, of the pass
#pragma unroll
        for (int j = 0; j < (BINS + kSortBlock - 1) / kSortBlock; ++j) {
            const int d = threadIdx.x + j * kSortBlock;
            uint32_t total, total_g;
            const uint32_t ex = block_excl_sum<kSortBlock>(my_tot[j], total, s_tmp);
            const uint32_t gtot = d < BINS ? bin_total[d] : 0u;
            const uint32_t exg = block_excl_sum<kSortBlock>(gtot, total_g, s_tmp);
            if (d < BINS) {
                s_start[d] = running + ex;
                s_dst[d] = running_g + exg + row_prefix[(size_t)d * stride + tile];
            }
            running += total;
            running_g += total_g;
        }
        if (DROP && threadIdx.x == 0) {
            s_tile_n = running;
            // the live count of the following passes: every block knows it, tile 0 writes it
            if (tile == 0u) *live_out = running_g;
        }
    }
    __syncthreads();
    uint32_t slot[ITEMS];   // LDS slot of each item, ~0u for an item that takes no part
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const uint32_t idx = base + it * kWave + lane;
        slot[it] = ~0u;
        if (idx < n && !(DROP && key[it] == drop_key)) {
            const uint32_t d = (key[it] >> shift) & (BINS - 1);
            slot[it] = s_start[d] + s_cnt[w][d] + rank[it];
            s_key[slot[it]] = key[it];
            s_val[slot[it]] = val[it];
        }
    }
    __syncthreads();
    // V2: the second values are requested now and arrive while the pairs
    // are written; they then take the value slots in LDS (no extra LDS, so
    // the occupancy of the pair-only passes is kept).
    uint32_t a2[V2 ? ITEMS : 1];
    if constexpr (V2) {
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint32_t idx = base + it * kWave + lane;
            a2[it] = idx < n ? ain[idx] : 0u;
        }
    }
    uint32_t tile_n;
    if constexpr (DROP) tile_n = s_tile_n;
    else tile_n = (n - tile * TILE) < (uint32_t)TILE ? (n - tile * TILE) : (uint32_t)TILE;
    for (uint32_t j = threadIdx.x; j < tile_n; j += kSortBlock) {
        const uint32_t k = s_key[j];
        const uint32_t d = (k >> shift) & (BINS - 1);
        const uint32_t dst = s_dst[d] + (j - s_start[d]);
        kout[dst] = k;
        vout[dst] = s_val[j];
    }
    if constexpr (V2) {
        __syncthreads();
#pragma unroll
        for (int it = 0; it < ITEMS; ++it)
            if (slot[it] != ~0u) s_val[slot[it]] = a2[it];
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < tile_n; j += kSortBlock) {
            const uint32_t d = (s_key[j] >> shift) & (BINS - 1);
            aout[s_dst[d] + (j - s_start[d])] = s_val[j];
        }
    }
}

template <int D, int ITEMS>
static void sort_pass(const uint32_t* kin, const uint32_t* vin, uint32_t* kout, uint32_t* vout,
                      const uint32_t* ain, uint32_t* aout, const uint32_t* n_dev, int64_t n_bound, int shift,
                      uint32_t* counts, bool drop, uint32_t drop_key, uint32_t* live_out, hipStream_t s) {
    const size_t tiles = tiles_for(ITEMS, n_bound);
    const uint32_t stride = (uint32_t)tiles + 1;
    uint32_t* totals = counts + ((size_t)1 << D) * stride;
    {
        ProfScope p(kStSortUpsweep, s);
        if (drop)
            hipLaunchKernelGGL((k_radix_upsweep<D, ITEMS, true>), dim3((unsigned)tiles), dim3(kSortBlock), 0, s,
                               kin, n_dev, (uint32_t)n_bound, shift, counts, stride, drop_key);
        else
            hipLaunchKernelGGL((k_radix_upsweep<D, ITEMS, false>), dim3((unsigned)tiles), dim3(kSortBlock), 0, s,
                               kin, n_dev, (uint32_t)n_bound, shift, counts, stride, drop_key);
    }
    {
        ProfScope p(kStSortScan, s);
        hipLaunchKernelGGL(k_scan_rows, dim3(1u << D), dim3(kSortBlock), 0, s, counts, stride, n_dev,
                           (uint32_t)n_bound, (uint32_t)(kSortBlock * ITEMS), totals);
    }
    {
        ProfScope p(kStSortDownsweep, s);
        const size_t grid = (tiles + 8 * kXcdGroup - 1) / (8 * kXcdGroup) * (8 * kXcdGroup);
        auto go = [&](auto kern, uint32_t* lo) {
            hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kSortBlock), 0, s, kin, vin, kout, vout, ain, aout,
                               n_dev, (uint32_t)n_bound, shift, counts, stride, totals, drop_key, lo);
        };
        if (drop)
            go(k_radix_downsweep<D, ITEMS, 2>, live_out);
        else if (ain)
            go(k_radix_downsweep<D, ITEMS, 1>, nullptr);
        else
            go(k_radix_downsweep<D, ITEMS, 0>, nullptr);
    }
}

using PassFn = void (*)(const uint32_t*, const uint32_t*, uint32_t*, uint32_t*, const uint32_t*, uint32_t*,
                        const uint32_t*, int64_t, int, uint32_t*, bool, uint32_t, uint32_t*, hipStream_t);

static PassFn pass_fn(int digit, int items) {
#define INPC_CASE(D, I) \
    if (digit == D && items == I) return &sort_pass<D, I>;
    INPC_CASE(7, 8) INPC_CASE(7, 16)
    INPC_CASE(8, 8) INPC_CASE(8, 16)
    INPC_CASE(9, 8) INPC_CASE(9, 16)
    INPC_CASE(10, 8)
    INPC_CASE(11, 8) INPC_CASE(11, 16)
#undef INPC_CASE
    return nullptr;
}

// Pass 0 reads (kin, vin) and writes (ka, va); later passes alternate
// (ka, va) -> (kb, vb) -> (ka, va) ...  (kin, vin) may alias (kb, vb).
// live_out != nullptr: pass 0 leaves out every key equal to drop_key and
// writes the number of kept keys to *live_out, which bounds the later passes
// (the sorted result is that many keys long); it requires a second value
// per key (ain, alternating aa / ab like the values; three distinct arrays),
// which is permuted with the pairs.
void launch_radix_sort(int digit, int items, int bits, const uint32_t* kin, const uint32_t* vin,
                       uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb,
                       const uint32_t* n_dev, int64_t n_bound, uint32_t* counts, hipStream_t s,
                       uint32_t drop_key, uint32_t* live_out, const uint32_t* ain, uint32_t* aa, uint32_t* ab) {
    const int passes = radix_passes(digit, bits);
    if (n_bound == 0 || passes == 0) {
        // nothing sorted: every key stays where it is (keys to drop included)
        if (live_out) launch_fill_u32(live_out, (uint32_t)n_bound, 1, s);
        return;
    }
    PassFn fn = pass_fn(digit, items);
    const uint32_t* ki = kin;
    const uint32_t* vi = vin;
    const uint32_t* ai = ain;
    uint32_t *ko = ka, *vo = va, *ao = aa;
    for (int p = 0; p < passes; ++p) {
        const bool drop = p == 0 && live_out != nullptr;
        fn(ki, vi, ko, vo, ai, ai ? ao : nullptr, p > 0 && live_out ? live_out : n_dev, n_bound, p * digit, counts,
           drop, drop_key, drop ? live_out : nullptr, s);
        ki = ko;
        vi = vo;
        ai = ai ? ao : nullptr;
        ko = (ko == ka) ? kb : ka;
        vo = (vo == va) ? vb : va;
        ao = (ao == aa) ? ab : aa;
    }
}

bool sort_valid(int digit, int items) { return pass_fn(digit, items) != nullptr; }

// ------------------------------------------------------------ pixel ranges
// One thread per group of kRangeGroup consecutive sorted keys (read with
// 16-byte loads) and the key in front of the group: every position i whose
// key differs from the one before starts the range of key[i] and ends the
// range of key[i-1].  Bins without keys keep the [0, 0) the fill gave them.
constexpr int kRangeGroup = 8;

__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ keys,
                                                const uint32_t* __restrict__ m_dev,
                                                uint32_t m_bound, uint2* __restrict__ range,
                                                uint32_t* __restrict__ clear, int clear_words) {
    if (clear && blockIdx.x == 0 && (int)threadIdx.x < clear_words) clear[threadIdx.x] = 0u;
    const uint32_t m = live_count(m_dev, m_bound);
    const uint32_t i0 = (blockIdx.x * blockDim.x + threadIdx.x) * (uint32_t)kRangeGroup;
    if (i0 >= m) return;
    uint32_t k[kRangeGroup];
    if (i0 + kRangeGroup <= m) {
        const uint4 a = reinterpret_cast<const uint4*>(keys + i0)[0];
        const uint4 b = reinterpret_cast<const uint4*>(keys + i0)[1];
        k[0] = a.x; k[1] = a.y; k[2] = a.z; k[3] = a.w;
        k[4] = b.x; k[5] = b.y; k[6] = b.z; k[7] = b.w;
    } else {
#pragma unroll
        for (int j = 0; j < kRangeGroup; ++j) k[j] = i0 + j < m ? keys[i0 + j] : 0u;
    }
    uint32_t prev = i0 > 0 ? keys[i0 - 1] : 0u;
#pragma unroll
    for (int j = 0; j < kRangeGroup; ++j) {
        const uint32_t i = i0 + (uint32_t)j;
        if (i < m) {
            if (i == 0u || k[j] != prev) {
                range[k[j]].x = i;
                if (i > 0u) range[prev].y = i;
            }
            if (i + 1u == m) range[k[j]].y = m;
            prev = k[j];
        }
    }
}

constexpr int kOrderWords = 66;   // class counts, class cursors (tile order)

void launch_ranges(const uint32_t* pkey_sorted, const uint32_t* m_dev, int64_t m_bound,
                   int64_t n_pixels, uint2* range, bool cleared, uint32_t* order_tmp, hipStream_t s) {
    if (!cleared) launch_fill_u32(reinterpret_cast<uint32_t*>(range), 0u, (size_t)n_pixels * 2, s);
    if (m_bound == 0) {
        if (order_tmp) launch_fill_u32(order_tmp, 0u, kOrderWords, s);
        return;
    }
    const int64_t groups = (m_bound + kRangeGroup - 1) / kRangeGroup;
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, s, pkey_sorted, m_dev,
                       (uint32_t)m_bound, range, order_tmp, order_tmp ? kOrderWords : 0);
}

// ------------------------------------------------------------ tile order
// Blocks are dispatched in index order, so a heavy tile launched late
// becomes the tail of a blend launch.  perm lists the tiles by descending
// size class (class = bit length of the entry count), so the heaviest tiles
// start first.  The order inside a class is arbitrary (atomics): every tile
// is blended on its own, so results do not depend on it.  Two kernels: a
// class histogram (one global atomic per block and class), and the
// placement, where every block derives the class starts from the histogram
// and reserves its slots with one atomic per class.  The counters are
// cleared by the ranges kernel.
constexpr int kOrderClasses = 33;
static_assert(2 * kOrderClasses <= kOrderWords, "order counters");

__device__ __forceinline__ int size_class(const uint2 rg) {
    const uint32_t n = rg.y - rg.x;
    return n ? 32 - __clz(n) : 0;
}

__global__ __launch_bounds__(256) void k_order_hist(const uint2* __restrict__ range, int64_t n_tiles,
                                                    uint32_t* __restrict__ cls_cnt) {
    __shared__ uint32_t h[kOrderClasses];
    for (int i = threadIdx.x; i < kOrderClasses; i += 256) h[i] = 0u;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n_tiles) atomicAdd(&h[size_class(range[t])], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < kOrderClasses; i += 256)
        if (h[i]) atomicAdd(&cls_cnt[i], h[i]);
}

// cls_cnt: class counts (read); cls_next: per-class cursors from 0 (advanced).
__global__ __launch_bounds__(256) void k_order_place(const uint2* __restrict__ range, int64_t n_tiles,
                                                     const uint32_t* __restrict__ cls_cnt,
                                                     uint32_t* __restrict__ cls_next, uint32_t* __restrict__ perm) {
    __shared__ uint32_t h[kOrderClasses];
    __shared__ uint32_t base[kOrderClasses];
    for (int i = threadIdx.x; i < kOrderClasses; i += 256) h[i] = 0u;
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int c = 0;
    uint32_t local = 0;
    if (t < n_tiles) {
        c = size_class(range[t]);
        local = atomicAdd(&h[c], 1u);
    }
    __syncthreads();
    // Lane k of the first wave serves class k: the reservations are issued
    // together (one round trip, not one per class), and class k starts
    // after all larger classes (a suffix sum of the class counts).
    if (threadIdx.x < kWave) {
        const int k = threadIdx.x;
        const bool cls = k < kOrderClasses;
        const uint32_t mine = cls ? h[k] : 0u;
        const uint32_t got = mine ? atomicAdd(&cls_next[k], mine) : 0u;
        uint32_t suf = cls ? cls_cnt[k] : 0u;   // inclusive suffix sum over classes >= k
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t o = __shfl_down(suf, d);
            if (k + d < kWave) suf += o;
        }
        if (cls) base[k] = mine ? (suf - cls_cnt[k]) + got : 0u;
    }
    __syncthreads();
    if (t < n_tiles) perm[base[c] + local] = (uint32_t)t;
}

void launch_tile_order(const uint2* range, int64_t n_tiles, uint32_t* order_tmp, uint32_t* perm, hipStream_t s) {
    if (n_tiles == 0) return;
    const unsigned blocks = (unsigned)((n_tiles + 255) / 256);
    hipLaunchKernelGGL(k_order_hist, dim3(blocks), dim3(256), 0, s, range, n_tiles, order_tmp);
    hipLaunchKernelGGL(k_order_place, dim3(blocks), dim3(256), 0, s, range, n_tiles, order_tmp,
                       order_tmp + kOrderClasses, perm);
}

}  // namespace inpc
