// Shared device-side definitions of the gfx950 rasterizer kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

namespace inpc {

constexpr int kWave = 64;

// Device copy of one view (written into the workspace by k_upload_views).
struct alignas(16) GpuView {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    float near_p, far_p;
    int32_t W, H;
    int64_t point_offset;   // first point of this view in the point arrays
    int64_t vpoint_offset;  // first view point (row of the per-view-point arrays)
    int64_t point_count;
    int64_t pixel_offset;   // first packed pixel
    int64_t tile_offset;    // first blend tile
    int64_t tiles_x;        // blend tiles per image row
    int64_t attr_offset;    // feature / opacity row of this view's first point
};
static_assert(sizeof(GpuView) == 144, "GpuView layout");

// Per view point record produced by the projection:
//   ax, ay  fractional offsets of (u-0.5, v-0.5) from the 2x2 anchor pixel,
//   opa     the point's opacity alpha_h,
//   anc     (x0+1) | (y0+1) << 14 | corner mask << 28, 0 when the point emits
//           no splat.  Corner c = 2*dy + dx covers pixel (x0+dx, y0+dy).
struct alignas(16) PointRec {
    float ax, ay, opa;
    uint32_t anc;
};

constexpr uint32_t kCulledKey = 0xFFFFFFFFu;
constexpr uint32_t kVpMask = 0x0FFFFFFFu;   // view point index bits of a depth-sort value

__device__ __forceinline__ int anc_x0(uint32_t a) { return (int)(a & 0x3FFFu) - 1; }
__device__ __forceinline__ int anc_y0(uint32_t a) { return (int)((a >> 14) & 0x3FFFu) - 1; }
__device__ __forceinline__ uint32_t anc_mask(uint32_t a) { return a >> 28; }

// Binary search: last view whose ``field`` start is <= x.
template <typename Getter>
__device__ __forceinline__ int find_view(const GpuView* __restrict__ views, int n_views, int64_t x,
                                         Getter get) {
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (get(views[mid]) <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << __lane_id()) - 1ull;
}

// Inclusive prefix sum over a wave64.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
    const int l = __lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (l >= o) x += y;
    }
    return x;
}

// Exclusive prefix sum over the block; s_tmp holds BLOCK/64 words.  Every
// thread of the block must call it.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t x, uint32_t& total, uint32_t* s_tmp) {
    constexpr int W = BLOCK / kWave;
    const uint32_t inc = wave_incl_sum(x);
    const int w = threadIdx.x / kWave;
    if (__lane_id() == kWave - 1) s_tmp[w] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        const uint32_t v = s_tmp[i];
        base += (i < w) ? v : 0u;
        tot += v;
    }
    __syncthreads();
    total = tot;
    return base + inc - x;
}

// Lanes of the wave whose ``digit`` (D low bits) equals this lane's, among
// the lanes with ``valid`` set.  D ballots, one per digit bit.
template <int D>
__device__ __forceinline__ uint64_t match_digit(uint32_t digit, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < D; ++b) {
        const bool bit = (digit >> b) & 1u;
        const uint64_t ones = __ballot(bit);
        m &= bit ? ones : ~ones;
    }
    return m;
}

// Feature row loads (float32 or bfloat16 storage, widened to float32).
// float32 -> bfloat16 bits, round to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0u;
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}

template <int F>
__device__ __forceinline__ void load_row(const float* __restrict__ row, float (&c)[F]) {
    if constexpr (F % 4 == 0) {
#pragma unroll
        for (int i = 0; i < F / 4; ++i) {
            const float4 v = reinterpret_cast<const float4*>(row)[i];
            c[4 * i] = v.x; c[4 * i + 1] = v.y; c[4 * i + 2] = v.z; c[4 * i + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < F; ++i) c[i] = row[i];
    }
}

template <int F>
__device__ __forceinline__ void load_row(const __hip_bfloat16* __restrict__ row_, float (&c)[F]) {
    const uint16_t* row = reinterpret_cast<const uint16_t*>(row_);
    if constexpr (F % 8 == 0) {
#pragma unroll
        for (int i = 0; i < F / 8; ++i) {
            const uint4 v = reinterpret_cast<const uint4*>(row)[i];
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                c[8 * i + 2 * j] = __uint_as_float(w[j] << 16);
                c[8 * i + 2 * j + 1] = __uint_as_float(w[j] & 0xFFFF0000u);
            }
        }
    } else if constexpr (F % 4 == 0) {
#pragma unroll
        for (int i = 0; i < F / 4; ++i) {
            const uint2 v = reinterpret_cast<const uint2*>(row)[i];
            c[4 * i] = __uint_as_float(v.x << 16);
            c[4 * i + 1] = __uint_as_float(v.x & 0xFFFF0000u);
            c[4 * i + 2] = __uint_as_float(v.y << 16);
            c[4 * i + 3] = __uint_as_float(v.y & 0xFFFF0000u);
        }
    } else {
#pragma unroll
        for (int i = 0; i < F; ++i) c[i] = bf16_to_f32(row[i]);
    }
}

template <int F>
__device__ __forceinline__ void store_row(float* __restrict__ row, const float (&c)[F]) {
    if constexpr (F % 4 == 0) {
#pragma unroll
        for (int i = 0; i < F / 4; ++i)
            reinterpret_cast<float4*>(row)[i] = make_float4(c[4 * i], c[4 * i + 1], c[4 * i + 2], c[4 * i + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < F; ++i) row[i] = c[i];
    }
}

// Bilinear factor of corner c (Section 3.4, Eq. 6) in float32, in the same
// operation order as the projection defines it: w_x = ax for the right
// column, 1 - ax for the left one.
__device__ __forceinline__ void corner_factors(float ax, float ay, int c, float& wx, float& wy) {
#pragma clang fp contract(off)
    wx = (c & 1) ? ax : 1.0f - ax;
    wy = (c & 2) ? ay : 1.0f - ay;
}

// Splat opacity alpha = opa * wx * wy and its complement 1 - alpha.  The
// complement is formed from the exact product (two error-free products via
// fma), so it keeps full relative precision when alpha is close to one.
__device__ __forceinline__ void splat_alpha(float opa, float wx, float wy, float& alpha, float& om) {
#pragma clang fp contract(off)
    const float w_hi = wx * wy;
    const float w_lo = __builtin_fmaf(wx, wy, -w_hi);
    alpha = opa * w_hi;
    const float om1 = __builtin_fmaf(-opa, w_hi, 1.0f);
    om = __builtin_fmaf(-opa, w_lo, om1);
}

// Block index -> logical index so that each XCD (blocks are dealt to the 8
// XCDs round-robin) receives one contiguous range of logical blocks.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb) {
    const uint32_t q = nb >> 3, r = nb & 7u;
    const uint32_t x = b & 7u, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

}  // namespace inpc
