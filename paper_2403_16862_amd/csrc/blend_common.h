// Device helpers shared by the blend kernels (forward, backward, point
// reduction): pixel tiling, feature-row access and the grouped transmittance
// step.
#pragma once

#include "internal.h"

namespace inpc {

// Pixel owned by this lane.  A wave covers a WXP x (64/L/WXP) pixel tile with
// L consecutive lanes per pixel; a block of 4 waves covers 2x2 wave tiles.
// Blocks are dealt to XCDs so that each XCD works on one contiguous band of
// tiles (neighbouring tiles share the points on their borders).
struct TileCoord {
    const GpuView* V;
    int64_t q;   // packed pixel index
    bool inside;
};

template <int WXP, int L>
__device__ __forceinline__ TileCoord tile_pixel(const GpuView* __restrict__ views, int n_views) {
    constexpr int WYP = kWave / L / WXP;
    const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int v = n_views == 1 ? 0
                               : find_view(views, n_views, (int64_t)t,
                                           [](const GpuView& g) { return g.tile_offset; });
    const GpuView* V = views + v;
    const int64_t lt = (int64_t)t - V->tile_offset;
    const int tx = (int)(lt % V->tiles_x), ty = (int)(lt / V->tiles_x);
    const int w = threadIdx.x / kWave, pl = __lane_id() / L;
    const int x = tx * (2 * WXP) + (w & 1) * WXP + (pl % WXP);
    const int y = ty * (2 * WYP) + (w >> 1) * WYP + (pl / WXP);
    TileCoord tc;
    tc.V = V;
    tc.inside = x < V->W && y < V->H;
    tc.q = V->pixel_offset + (int64_t)y * V->W + x;
    return tc;
}

// Feature row of a point, widened to float32.  DYN: runtime F (Fd) <= FM.
template <typename FT, int FM, bool DYN>
__device__ __forceinline__ void feat_row(const FT* __restrict__ feat, int64_t p, int Fd, float (&c)[FM]) {
    if constexpr (!DYN) {
        load_row<FM>(feat + p * FM, c);
    } else {
        const FT* row = feat + p * Fd;
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            if (f < Fd) {
                if constexpr (sizeof(FT) == 4) c[f] = reinterpret_cast<const float*>(row)[f];
                else c[f] = bf16_to_f32(reinterpret_cast<const uint16_t*>(row)[f]);
            } else {
                c[f] = 0.0f;
            }
        }
    }
}

template <int FM, bool DYN>
__device__ __forceinline__ void f32_row(const float* __restrict__ base, int64_t r, int Fd, float (&c)[FM]) {
    if constexpr (!DYN) {
        load_row<FM>(base + r * FM, c);
    } else {
        const float* row = base + r * Fd;
#pragma unroll
        for (int f = 0; f < FM; ++f) c[f] = f < Fd ? row[f] : 0.0f;
    }
}

template <int FM, bool DYN>
__device__ __forceinline__ void f32_store(float* __restrict__ base, int64_t r, int Fd, const float (&c)[FM]) {
    if constexpr (!DYN) {
        store_row<FM>(base + r * FM, c);
    } else {
        float* row = base + r * Fd;
#pragma unroll
        for (int f = 0; f < FM; ++f)
            if (f < Fd) row[f] = c[f];
    }
}

// One group step of the front-to-back recurrence for the L lanes of a pixel
// (lane ``sub`` holds splat base+sub, or nothing if !valid: om = 1).
// Inputs: T before the group, the lane's 1 - alpha.  Outputs: the lane's T
// before/after its splat, whether it is blended (the first splat always is;
// any other one iff the transmittance before it is still >= tau, which is
// the "apply, then stop once T < tau" rule), and the T after the group with
// a flag telling whether the pixel terminated inside it.
struct GroupStep {
    float tb, ta;
    bool blended;
    float t_next;
    bool done;
};

template <int L>
__device__ __forceinline__ GroupStep group_step(float T, float om, bool valid, bool first, float tau,
                                                int sub) {
    float pin = om;
#pragma unroll
    for (int d = 1; d < L; d <<= 1) {
        const float t = __shfl_up(pin, d, L);
        if (sub >= d) pin *= t;
    }
    float pex = __shfl_up(pin, 1, L);
    if (sub == 0) pex = 1.0f;
    GroupStep g;
    g.tb = T * pex;
    g.ta = T * pin;
    g.blended = valid && (first || g.tb >= tau);
    const bool term = g.blended && g.ta < tau;
    const int gbase = __lane_id() - sub;
    const uint64_t tm = __ballot(term);
    const uint32_t mine = (uint32_t)((tm >> gbase) & ((L == 64) ? ~0ull : ((1ull << L) - 1ull)));
    if (mine) {
        g.t_next = __shfl(g.ta, __ffs(mine) - 1, L);
        g.done = true;
    } else {
        g.t_next = __shfl(g.ta, L - 1, L);
        g.done = false;
    }
    return g;
}

// Calls body.template operator()<FM, DYN>() for the compiled feature widths.
template <typename Body>
__host__ static bool dispatch_f(int F, Body&& body) {
    switch (F) {
        case 1: body.template operator()<1, false>(); return true;
        case 2: body.template operator()<2, false>(); return true;
        case 3: body.template operator()<3, false>(); return true;
        case 4: body.template operator()<4, false>(); return true;
        case 8: body.template operator()<8, false>(); return true;
        case 16: body.template operator()<16, false>(); return true;
        case 32: body.template operator()<32, false>(); return true;
        default: break;
    }
    if (F < 1 || F > 64) return false;
    if (F <= 16) body.template operator()<16, true>();
    else if (F <= 32) body.template operator()<32, true>();
    else body.template operator()<64, true>();
    return true;
}

// Blend shapes: lanes per pixel and wave-tile width in pixels.
template <typename Body>
__host__ static void dispatch_shape(int shape, Body&& body) {
    switch (shape) {
        case 1: body.template operator()<8, 2>(); break;
        case 2: body.template operator()<4, 4>(); break;
        case 3: body.template operator()<4, 8>(); break;
        case 4: body.template operator()<2, 16>(); break;
        default: body.template operator()<8, 1>(); break;
    }
}

}  // namespace inpc
