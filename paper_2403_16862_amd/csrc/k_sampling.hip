// Point sampling from the probability octree (Section 3.2, Eq. 4; Appendix
// A.4) and the per-leaf probability updates (Section 3.1, Eq. 2 and Eq. 3)
// for gfx950.
//
// Every decision is exact and reproducible: the re-weighted probabilities
// are float32 operations in a fixed order (no contraction), the multinomial
// draw inverts an integer CDF of fixed-point weights, random numbers come
// from the counter-based Philox4x64-10 generator (Salmon et al., SC 2011)
// keyed by the caller's seed, and per-leaf reductions use integer atomics
// only (their results do not depend on the order of the updates).
#include "internal.h"

namespace inpc {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull, kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull, kPhiloxW1 = 0xBB67AE8584CAA73Bull;
constexpr int kScanBlock = 256, kScanItems = 8, kScanTile = kScanBlock * kScanItems;

__device__ __forceinline__ void philox4x64(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(kPhiloxM0, c[0]), lo0 = kPhiloxM0 * c[0];
        const uint64_t hi1 = __umul64hi(kPhiloxM1, c[2]), lo1 = kPhiloxM1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
}

__device__ __forceinline__ float unit24(uint64_t x) { return (float)(x >> 40) * 0x1.0p-24f; }

__device__ __forceinline__ float leaf_edge(float root, int level) { return ldexpf(root, -level); }

__device__ __forceinline__ int clamp_level(int l) { return l < 0 ? 0 : (l > 31 ? 31 : l); }

__device__ __forceinline__ void to_view(const SampleCam& C, float x, float y, float z, float& xc, float& yc,
                                        float& zc) {
#pragma clang fp contract(off)
    xc = ((C.R[0] * x + C.R[1] * y) + C.R[2] * z) + C.t[0];
    yc = ((C.R[3] * x + C.R[4] * y) + C.R[5] * z) + C.t[1];
    zc = ((C.R[6] * x + C.R[7] * y) + C.R[8] * z) + C.t[2];
}

// The cube is visible unless all 8 corners lie outside one of the six
// frustum half-spaces (near, far, u = 0, u = W, v = 0, v = H).
__device__ __forceinline__ bool cube_visible(const SampleCam& C, float cx0, float cy0, float cz0, float h) {
#pragma clang fp contract(off)
    uint32_t inside = 0;   // bit k: some corner is inside half-space k
    const float Wf = (float)C.W, Hf = (float)C.H;
#pragma unroll
    for (int corner = 0; corner < 8; ++corner) {
        const float x = cx0 + ((corner & 1) ? h : -h);
        const float y = cy0 + ((corner & 2) ? h : -h);
        const float z = cz0 + ((corner & 4) ? h : -h);
        float xc, yc, zc;
        to_view(C, x, y, z, xc, yc, zc);
        const float us = C.fx * xc + C.cx * zc;
        const float vs = C.fy * yc + C.cy * zc;
        inside |= (zc - C.near_p > 0.0f) ? 1u : 0u;
        inside |= (C.far_p - zc > 0.0f) ? 2u : 0u;
        inside |= (us > 0.0f) ? 4u : 0u;
        inside |= (Wf * zc - us > 0.0f) ? 8u : 0u;
        inside |= (vs > 0.0f) ? 16u : 0u;
        inside |= (Hf * zc - vs > 0.0f) ? 32u : 0u;
    }
    return inside == 63u;
}

__device__ __forceinline__ bool point_in_view(const SampleCam& C, float x, float y, float z) {
#pragma clang fp contract(off)
    float xc, yc, zc;
    to_view(C, x, y, z, xc, yc, zc);
    if (!(zc > C.near_p && zc < C.far_p)) return false;
    const float u = C.fx * (xc / zc) + C.cx;
    const float v = C.fy * (yc / zc) + C.cy;
    return u >= 0.0f && u < (float)C.W && v >= 0.0f && v < (float)C.H;
}

__device__ __forceinline__ float place(float c, float frac, float edge) {
#pragma clang fp contract(off)
    return c + (frac - 0.5f) * edge;
}

// ------------------------------------------------ re-weighting (Eq. 4)
__global__ __launch_bounds__(256) void k_leaf_weight(const float* __restrict__ centre,
                                                     const int32_t* __restrict__ level,
                                                     const float* __restrict__ prob, int64_t n_leaves,
                                                     float root, float tau_d, LevelTable lt, SampleCam cam,
                                                     int view, float* __restrict__ phat,
                                                     uint32_t* __restrict__ max_bits) {
#pragma clang fp contract(off)
    __shared__ uint32_t s_max[256 / kWave];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float ph = 0.0f;
    if (i < n_leaves) {
        const int l = clamp_level(level[i]);
        const float p = prob[i];
        if (view) {
            const float x = centre[3 * i], y = centre[3 * i + 1], z = centre[3 * i + 2];
            const float h = leaf_edge(root, l) * 0.5f;
            if (cube_visible(cam, x, y, z, h)) {
                float xc, yc, zc;
                to_view(cam, x, y, z, xc, yc, zc);
                float d = fabsf(zc - cam.near_p) / cam.far_p;
                d = fmaxf(d, tau_d);
                ph = p / (d * lt.f[l]);
            }
        } else {
            ph = p / lt.f[l];
        }
        phat[i] = ph;
    }
    // re-weighted probabilities are >= 0, so their float bits order like the values
    uint32_t m = __float_as_uint(ph);
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(m, d);
        m = o > m ? o : m;
    }
    if (__lane_id() == 0) s_max[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = s_max[0];
        for (int w = 1; w < 256 / kWave; ++w) b = s_max[w] > b ? s_max[w] : b;
        atomicMax(max_bits, b);
    }
}

// Fixed-point weight of a re-weighted probability: with the largest value
// m < 2^e, w = floor(p_hat * 2^(38 - e)) (exact in float64).
struct PhatWeight {
    const float* phat;
    const uint32_t* max_bits;
    __device__ __forceinline__ uint64_t operator()(int64_t i, int shift) const {
        return (uint64_t)floor(ldexp((double)phat[i], shift));
    }
    __device__ __forceinline__ int prepare() const {
        const float m = __uint_as_float(*max_bits);
        int e = 0;
        (void)frexpf(m, &e);
        return 38 - e;
    }
};

struct CountWeight {
    const uint32_t* counts;
    __device__ __forceinline__ uint64_t operator()(int64_t i, int) const { return (uint64_t)counts[i]; }
    __device__ __forceinline__ int prepare() const { return 0; }
};

__device__ __forceinline__ uint64_t wave_incl_sum_u64(uint64_t x) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t y = __shfl_up(x, d);
        if (__lane_id() >= d) x += y;
    }
    return x;
}

// Block-wide exclusive scan of one uint64 per thread; returns the prefix and
// the block total.
__device__ __forceinline__ uint64_t block_excl_u64(uint64_t x, uint64_t& total, uint64_t* s_w) {
    const uint64_t inc = wave_incl_sum_u64(x);
    const int w = threadIdx.x / kWave;
    if (__lane_id() == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint64_t base = 0, tot = 0;
    for (int k = 0; k < kScanBlock / kWave; ++k) {
        if (k < w) base += s_w[k];
        tot += s_w[k];
    }
    __syncthreads();
    total = tot;
    return base + inc - x;
}

// Inclusive prefix sums of 64-bit weights: tile sums, one-block scan of the
// tile sums, then per-tile scan plus tile offset.
template <typename Wt>
__global__ __launch_bounds__(kScanBlock) void k_wscan_tiles(Wt wt, int64_t n, uint64_t* __restrict__ tile_sum) {
    __shared__ uint64_t s_w[kScanBlock / kWave];
    const int shift = wt.prepare();
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += wt(base + k, shift);
    uint64_t total;
    (void)block_excl_u64(s, total, s_w);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_wscan_top(uint64_t* __restrict__ tile_sum, int64_t n_tiles) {
    __shared__ uint64_t s_w[kScanBlock / kWave];
    uint64_t running = 0;
    for (int64_t b = 0; b < n_tiles; b += kScanBlock) {
        const int64_t i = b + threadIdx.x;
        const uint64_t x = i < n_tiles ? tile_sum[i] : 0ull;
        uint64_t total;
        const uint64_t ex = block_excl_u64(x, total, s_w);
        if (i < n_tiles) tile_sum[i] = running + ex;
        running += total;
    }
}

template <typename Wt>
__global__ __launch_bounds__(kScanBlock) void k_wscan_apply(Wt wt, int64_t n, const uint64_t* __restrict__ tile_off,
                                                            uint64_t* __restrict__ cdf) {
    __shared__ uint64_t s_w[kScanBlock / kWave];
    const int shift = wt.prepare();
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint64_t v[kScanItems];
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < n ? wt(base + k, shift) : 0ull;
        s += v[k];
    }
    uint64_t total;
    uint64_t run = tile_off[blockIdx.x] + block_excl_u64(s, total, s_w);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        run += v[k];
        if (base + k < n) cdf[base + k] = run;
    }
}

template <typename Wt>
static void weight_scan(Wt wt, int64_t n, uint64_t* tile_sum, uint64_t* cdf, hipStream_t s) {
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_wscan_tiles<Wt>, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, wt, n, tile_sum);
    hipLaunchKernelGGL(k_wscan_top, dim3(1), dim3(kScanBlock), 0, s, tile_sum, tiles);
    hipLaunchKernelGGL(k_wscan_apply<Wt>, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, wt, n,
                       (const uint64_t*)tile_sum, cdf);
}

// First leaf i with cdf[i] > t (t < cdf[n-1]).
__device__ __forceinline__ int64_t upper_bound_u64(const uint64_t* __restrict__ cdf, int64_t n, uint64_t t) {
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cdf[mid] > t) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Guide table of the inverse-CDF search: bucket b of 2^g holds the leaf
// upper_bound(cdf, T_b) with T_b = the draw target of the smallest 64-bit
// word whose top g bits are b (T_G = total).  Targets are monotone in the
// word, so the leaf of a word in bucket b lies in [guide[b], guide[b + 1]]
// and a binary search over that (short) range returns exactly the leaf of
// the search over the whole CDF.
__global__ __launch_bounds__(256) void k_guide(const uint64_t* __restrict__ cdf, int64_t n_leaves, int g,
                                               uint32_t* __restrict__ guide) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t G = (int64_t)1 << g;
    if (b > G) return;
    const uint64_t total = cdf[n_leaves - 1];
    const uint64_t tb = b == G ? total : __umul64hi((uint64_t)b << (64 - g), total);
    guide[b] = (uint32_t)upper_bound_u64(cdf, n_leaves, tb);
}

// The leaf drawn by the 64-bit word c0: the first with cdf > umul64hi(c0, total).
__device__ __forceinline__ int64_t guided_leaf(const uint64_t* __restrict__ cdf, const uint32_t* __restrict__ guide,
                                               int g, uint64_t c0, uint64_t total) {
    const uint64_t t = __umul64hi(c0, total);
    const uint64_t b = c0 >> (64 - g);
    int64_t lo = guide[b], hi = guide[b + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (cdf[mid] > t) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// ------------------------------------------- viewpoint-specific sampling
__global__ __launch_bounds__(256) void k_sample_view(const float* __restrict__ centre,
                                                     const int32_t* __restrict__ level, float root,
                                                     const uint64_t* __restrict__ cdf, int64_t n_leaves,
                                                     const uint32_t* __restrict__ guide, int g,
                                                     SampleCam cam, uint64_t seed0, uint64_t seed1,
                                                     int64_t n, int max_rounds, float* __restrict__ xyz,
                                                     int32_t* __restrict__ leaf_out,
                                                     unsigned long long* __restrict__ unresolved) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t total = cdf[n_leaves - 1];
    if (total == 0) {
        xyz[3 * s] = xyz[3 * s + 1] = xyz[3 * s + 2] = __uint_as_float(0x7FC00000u);
        leaf_out[s] = -1;
        atomicAdd(unresolved, 1ull);
        return;
    }
    const int rounds = max_rounds > 0 ? max_rounds : 1;
    float px = 0.0f, py = 0.0f, pz = 0.0f;
    int64_t leaf = 0;
    bool ok = false;
    for (int r = 0; r < rounds; ++r) {
        uint64_t c[4] = {(uint64_t)s, (uint64_t)r, 1ull, 0ull};
        philox4x64(c, seed0, seed1);
        leaf = guided_leaf(cdf, guide, g, c[0], total);
        const float e = leaf_edge(root, clamp_level(level[leaf]));
        px = place(centre[3 * leaf], unit24(c[1]), e);
        py = place(centre[3 * leaf + 1], unit24(c[2]), e);
        pz = place(centre[3 * leaf + 2], unit24(c[3]), e);
        if (max_rounds <= 0 || point_in_view(cam, px, py, pz)) {
            ok = true;
            break;
        }
    }
    xyz[3 * s] = px;
    xyz[3 * s + 1] = py;
    xyz[3 * s + 2] = pz;
    leaf_out[s] = (int32_t)leaf;
    if (!ok) atomicAdd(unresolved, 1ull);
}

// ---------------------------------------------------- global extraction
__global__ __launch_bounds__(256) void k_sample_count(const uint64_t* __restrict__ cdf, int64_t n_leaves,
                                                      const uint32_t* __restrict__ guide, int g,
                                                      uint64_t seed0, uint64_t seed1, int64_t n,
                                                      uint32_t* __restrict__ counts) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t total = cdf[n_leaves - 1];
    if (total == 0) return;
    uint64_t c[4] = {(uint64_t)s, 0ull, 2ull, 0ull};
    philox4x64(c, seed0, seed1);
    atomicAdd(&counts[guided_leaf(cdf, guide, g, c[0], total)], 1u);
}

// Van der Corput radical inverse in base b, digit by digit in float64.
__device__ __forceinline__ double radical_inverse(uint64_t k, uint32_t b) {
#pragma clang fp contract(off)
    const double inv = 1.0 / (double)b;
    double f = inv, r = 0.0;
    while (k > 0) {
        r = r + (double)(k % b) * f;
        k /= b;
        f = f * inv;
    }
    return r;
}

__global__ __launch_bounds__(256) void k_sample_expand(const float* __restrict__ centre,
                                                       const int32_t* __restrict__ level, float root,
                                                       const uint64_t* __restrict__ count_cdf, int64_t n_leaves,
                                                       int64_t n, float* __restrict__ xyz,
                                                       int32_t* __restrict__ leaf_out) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    if (count_cdf[n_leaves - 1] == 0) {
        xyz[3 * o] = xyz[3 * o + 1] = xyz[3 * o + 2] = __uint_as_float(0x7FC00000u);
        leaf_out[o] = -1;
        return;
    }
    const int64_t leaf = upper_bound_u64(count_cdf, n_leaves, (uint64_t)o);
    const uint64_t j = (uint64_t)o - (leaf > 0 ? count_cdf[leaf - 1] : 0ull);
    const float e = leaf_edge(root, clamp_level(level[leaf]));
    xyz[3 * o] = place(centre[3 * leaf], (float)radical_inverse(j + 1, 2), e);
    xyz[3 * o + 1] = place(centre[3 * leaf + 1], (float)radical_inverse(j + 1, 3), e);
    xyz[3 * o + 2] = place(centre[3 * leaf + 2], (float)radical_inverse(j + 1, 5), e);
    leaf_out[o] = (int32_t)leaf;
}

// ------------------------------------------- probability updates (Eq. 2, 3)
__device__ __forceinline__ uint32_t order_key(float x) {
    const uint32_t b = __float_as_uint(x);
    return (b >> 31) ? ~b : (b ^ 0x80000000u);
}
__device__ __forceinline__ float from_order_key(uint32_t k) {
    return __uint_as_float((k >> 31) ? (k ^ 0x80000000u) : ~k);
}

__global__ __launch_bounds__(256) void k_prob_minmax(const int32_t* __restrict__ leaf, const float* __restrict__ b,
                                                     int64_t n, int64_t n_leaves, uint32_t* __restrict__ kmax,
                                                     uint32_t* __restrict__ kmin) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t l = leaf[i];
    if (l < 0 || (int64_t)l >= n_leaves) return;
    const uint32_t k = order_key(b[i]);
    // The stored extrema only move outward, so a plain read (possibly of an
    // older value) that already bounds k makes the atomic unnecessary; most
    // samples of a leaf skip it.
    if (k > kmax[l]) atomicMax(&kmax[l], k);
    if (k < kmin[l]) atomicMin(&kmin[l], k);
}

__global__ __launch_bounds__(256) void k_prob_apply(const uint32_t* __restrict__ kmax,
                                                    const uint32_t* __restrict__ kmin, int64_t n_leaves,
                                                    float lambda_u, float* __restrict__ prob,
                                                    float* __restrict__ subdiv) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_leaves) return;
    float p = lambda_u * prob[i];
    float q = lambda_u * subdiv[i];
    const uint32_t hi = kmax[i];
    if (hi != 0u) {
        const float mx = from_order_key(hi), mn = from_order_key(kmin[i]);
        p = fmaxf(p, mx);
        q = fmaxf(q, mx - mn);
    }
    prob[i] = p;
    subdiv[i] = q;
}

// ------------------------------------------------------------ launchers
static unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

void launch_sample_weights(const float* centre, const int32_t* level, const float* prob, int64_t n_leaves,
                           float root, float tau_d, const LevelTable& lt, const SampleCam& cam, bool view,
                           float* phat, uint32_t* max_bits, uint64_t* tile_sum, uint64_t* cdf, hipStream_t s) {
    launch_fill_u32(max_bits, 0u, 1, s);
    hipLaunchKernelGGL(k_leaf_weight, dim3(blocks_for(n_leaves)), dim3(256), 0, s, centre, level, prob, n_leaves,
                       root, tau_d, lt, cam, view ? 1 : 0, phat, max_bits);
    weight_scan(PhatWeight{phat, max_bits}, n_leaves, tile_sum, cdf, s);
}

int guide_bits(int64_t n_leaves) {
    int g = 1;
    while (((int64_t)1 << g) < n_leaves) ++g;
    return g;
}

static void launch_guide(const uint64_t* cdf, int64_t n_leaves, uint32_t* guide, hipStream_t s) {
    const int g = guide_bits(n_leaves);
    hipLaunchKernelGGL(k_guide, dim3(blocks_for(((int64_t)1 << g) + 1)), dim3(256), 0, s, cdf, n_leaves, g, guide);
}

void launch_sample_view(const float* centre, const int32_t* level, float root, const uint64_t* cdf,
                        int64_t n_leaves, uint32_t* guide, const SampleCam& cam, uint64_t seed0, uint64_t seed1,
                        int64_t n, int max_rounds, float* xyz, int32_t* leaf, unsigned long long* unresolved,
                        hipStream_t s) {
    launch_fill_u32(reinterpret_cast<uint32_t*>(unresolved), 0u, 2, s);
    if (n == 0) return;
    launch_guide(cdf, n_leaves, guide, s);
    hipLaunchKernelGGL(k_sample_view, dim3(blocks_for(n)), dim3(256), 0, s, centre, level, root, cdf, n_leaves,
                       (const uint32_t*)guide, guide_bits(n_leaves), cam, seed0, seed1, n, max_rounds, xyz, leaf,
                       unresolved);
}

void launch_sample_global(const float* centre, const int32_t* level, float root, const uint64_t* cdf,
                          int64_t n_leaves, uint32_t* guide, uint64_t seed0, uint64_t seed1, int64_t n,
                          uint32_t* counts, uint64_t* tile_sum, uint64_t* count_cdf, float* xyz, int32_t* leaf,
                          hipStream_t s) {
    launch_fill_u32(counts, 0u, (size_t)n_leaves, s);
    if (n > 0) {
        launch_guide(cdf, n_leaves, guide, s);
        hipLaunchKernelGGL(k_sample_count, dim3(blocks_for(n)), dim3(256), 0, s, cdf, n_leaves,
                           (const uint32_t*)guide, guide_bits(n_leaves), seed0, seed1, n, counts);
    }
    weight_scan(CountWeight{counts}, n_leaves, tile_sum, count_cdf, s);
    if (n > 0)
        hipLaunchKernelGGL(k_sample_expand, dim3(blocks_for(n)), dim3(256), 0, s, centre, level, root,
                           (const uint64_t*)count_cdf, n_leaves, n, xyz, leaf);
}

void launch_prob_update(const int32_t* leaf, const float* b, int64_t n, int64_t n_leaves, float lambda_u,
                        float* prob, float* subdiv, uint32_t* kmax, uint32_t* kmin, hipStream_t s) {
    launch_fill_u32(kmax, 0u, (size_t)n_leaves, s);
    launch_fill_u32(kmin, 0xFFFFFFFFu, (size_t)n_leaves, s);
    if (n > 0)
        hipLaunchKernelGGL(k_prob_minmax, dim3(blocks_for(n)), dim3(256), 0, s, leaf, b, n, n_leaves, kmax, kmin);
    hipLaunchKernelGGL(k_prob_apply, dim3(blocks_for(n_leaves)), dim3(256), 0, s, (const uint32_t*)kmax,
                       (const uint32_t*)kmin, n_leaves, lambda_u, prob, subdiv);
}

}  // namespace inpc
