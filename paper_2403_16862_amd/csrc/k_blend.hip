// Per-pixel front-to-back blending (Eq. 1 with early termination, the
// BlendSortedSplats step of Algorithm 1), its backward, and the
// deterministic per-point gradient reduction (Appendix A.6) for gfx950.
//
// One lane owns one pixel and walks its depth-sorted splat list.  A wave
// covers a compact 2D pixel tile (wave_x x 64/wave_x) and a block 2x2 wave
// tiles, so the 2x2 footprint of most points falls into one block and the
// point records and feature rows it gathers are reused from the same L2.
// Blocks are dealt to XCDs so that each XCD works on one contiguous band of
// tiles.
#include "internal.h"

namespace inpc {

struct TileCoord {
    const GpuView* V;
    int64_t q;   // packed pixel index
    bool inside;
};

template <int WX>
__device__ __forceinline__ TileCoord tile_pixel(const GpuView* __restrict__ views, int n_views) {
    constexpr int WY = kWave / WX;
    const uint32_t t = xcd_remap(blockIdx.x, gridDim.x);
    const int v = n_views == 1 ? 0
                               : find_view(views, n_views, (int64_t)t,
                                           [](const GpuView& g) { return g.tile_offset; });
    const GpuView* V = views + v;
    const int64_t lt = (int64_t)t - V->tile_offset;
    const int tx = (int)(lt % V->tiles_x), ty = (int)(lt / V->tiles_x);
    const int w = threadIdx.x / kWave, lane = __lane_id();
    const int x = tx * (2 * WX) + (w & 1) * WX + (lane % WX);
    const int y = ty * (2 * WY) + (w >> 1) * WY + (lane / WX);
    TileCoord tc;
    tc.V = V;
    tc.inside = x < V->W && y < V->H;
    tc.q = V->pixel_offset + (int64_t)y * V->W + x;
    return tc;
}

// Feature row of view point vp, widened to float32.  DYN: runtime F <= FM.
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

// ------------------------------------------------------------ forward blend
template <typename FT, int FM, bool DYN, int WX>
__global__ __launch_bounds__(256) void k_blend_fwd(
    const GpuView* __restrict__ views, int n_views, const uint2* __restrict__ range,
    const uint32_t* __restrict__ ids, const PointRec* __restrict__ rec, const FT* __restrict__ feat,
    int Fd, float tau, float* __restrict__ image, float* __restrict__ t_final,
    PixelState* __restrict__ state, float* __restrict__ t_before) {
    const TileCoord tc = tile_pixel<WX>(views, n_views);
    if (!tc.inside) return;
    const int64_t pbase = tc.V->point_offset - tc.V->vpoint_offset;
    const uint2 r = range[tc.q];
    float C[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) C[f] = 0.0f;
    float T = 1.0f;
    uint32_t n = 0;
    for (uint32_t i = r.x; i < r.y; ++i) {
        const uint32_t id = ids[i];
        const uint32_t vp = id >> 2;
        const PointRec pr = rec[vp];
        float cf[FM];
        feat_row<FT, FM, DYN>(feat, pbase + vp, Fd, cf);
        float wx, wy, alpha, om;
        corner_factors(pr.ax, pr.ay, (int)(id & 3u), wx, wy);
        splat_alpha(pr.opa, wx, wy, alpha, om);
        const float ta = T * alpha;
#pragma unroll
        for (int f = 0; f < FM; ++f) C[f] = __builtin_fmaf(ta, cf[f], C[f]);
        if (t_before) t_before[i] = T;
        T = T * om;
        ++n;
        if (T < tau) break;
    }
    f32_store<FM, DYN>(image, tc.q, Fd, C);
    t_final[tc.q] = T;
    PixelState st;
    st.n_blended = n;
    st.pad0 = st.pad1 = st.pad2 = 0;
    state[tc.q] = st;
}

// ----------------------------------------------------------- backward blend
// Reverse walk over the blended splats k = n-1 .. 0 of a pixel with the
// scalar recurrence Y_k = alpha_k (g.c_k) + (1-alpha_k) Y_{k+1},
// Y_n = g_T, so that dL/dalpha_k = T_k ((g.c_k) - Y_{k+1}) and
// dL/dc_k = T_k alpha_k g.  T_k is the forward's own float32 value: stored
// by the forward blend (t_before, one word per blended splat), or, when
// ``rebuild_t`` is set, recomputed here by the same forward recurrence in a
// first walk over the pixel's splats (needs only the point records).
// Writes the per-splat record (dL/dalpha_k, T_k alpha_k) at splat id.
template <typename FT, int FM, bool DYN, int WX>
__global__ __launch_bounds__(256) void k_blend_bwd(
    const GpuView* __restrict__ views, int n_views, const uint2* __restrict__ range,
    const uint32_t* __restrict__ ids, const PointRec* __restrict__ rec, const FT* __restrict__ feat,
    int Fd, const PixelState* __restrict__ state, const float* __restrict__ g_img,
    const float* __restrict__ g_t, float* __restrict__ t_before, int rebuild_t,
    float2* __restrict__ frec) {
    const TileCoord tc = tile_pixel<WX>(views, n_views);
    if (!tc.inside) return;
    const uint32_t n = state[tc.q].n_blended;
    if (n == 0) return;
    const int64_t pbase = tc.V->point_offset - tc.V->vpoint_offset;
    const uint32_t start = range[tc.q].x;
    if (rebuild_t) {
        float T = 1.0f;
        for (uint32_t k = 0; k < n; ++k) {
            const uint32_t id = ids[start + k];
            const PointRec pr = rec[id >> 2];
            float wx, wy, alpha, om;
            corner_factors(pr.ax, pr.ay, (int)(id & 3u), wx, wy);
            splat_alpha(pr.opa, wx, wy, alpha, om);
            t_before[start + k] = T;
            T = T * om;
        }
    }
    float g[FM];
    f32_row<FM, DYN>(g_img, tc.q, Fd, g);
    // The scalar chain (g.c, alpha, 1 - alpha, Y) runs in float64 registers:
    // dL/dalpha is a difference of two nearly equal sums for most splats, and
    // float64 keeps that cancellation from eating the result.  Inputs and the
    // stored records stay float32.
    double Y = g_t ? (double)g_t[tc.q] : 0.0;
    for (int k = (int)n - 1; k >= 0; --k) {
        const uint32_t id = ids[start + k];
        const uint32_t vp = id >> 2;
        const PointRec pr = rec[vp];
        float cf[FM];
        feat_row<FT, FM, DYN>(feat, pbase + vp, Fd, cf);
        float wx, wy;
        corner_factors(pr.ax, pr.ay, (int)(id & 3u), wx, wy);
        const double alpha = (double)pr.opa * ((double)wx * (double)wy);
        const double om = 1.0 - alpha;
        double gc = 0.0;
#pragma unroll
        for (int f = 0; f < FM; ++f) gc = __builtin_fma((double)g[f], (double)cf[f], gc);
        const double Tk = (double)t_before[start + k];
        frec[id] = make_float2((float)(Tk * (gc - Y)), (float)(Tk * alpha));
        Y = __builtin_fma(alpha, gc, om * Y);
    }
}

// --------------------------------------------------- per-point reduction
// grad_opa[vp] = sum_c w_c dL/dalpha_c, grad_feat[vp] = sum_c T_c alpha_c g_{pixel(c)}
// over the existing corners c = 0..3 in ascending order; the per-splat
// records of a point are contiguous (ids 4vp .. 4vp+3), so this is a
// segmented reduction over the id-ordered splat records.  Non-blended
// splats hold zeros (the record array is cleared before the backward blend).
template <int FM, bool DYN>
__global__ __launch_bounds__(256) void k_point_reduce(
    const GpuView* __restrict__ views, int n_views, int64_t n_vp, const PointRec* __restrict__ rec,
    const float2* __restrict__ frec, const float* __restrict__ g_img, int Fd,
    float* __restrict__ grad_feat, float* __restrict__ grad_opa) {
    const int64_t vp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (vp >= n_vp) return;
    const PointRec pr = rec[vp];
    const uint32_t mask = anc_mask(pr.anc);
    // float64 accumulators: the (at most four) corner terms often cancel.
    double gf[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) gf[f] = 0.0;
    double go = 0.0;
    if (mask != 0u) {
        const int v = n_views == 1 ? 0
                                   : find_view(views, n_views, vp,
                                               [](const GpuView& g) { return g.vpoint_offset; });
        const GpuView& V = views[v];
        const int x0 = anc_x0(pr.anc), y0 = anc_y0(pr.anc);
        const float4 r01 = reinterpret_cast<const float4*>(frec)[2 * vp];
        const float4 r23 = reinterpret_cast<const float4*>(frec)[2 * vp + 1];
        const float da[4] = {r01.x, r01.z, r23.x, r23.z};
        const float ta[4] = {r01.y, r01.w, r23.y, r23.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!((mask >> c) & 1u)) continue;
            float wx, wy;
            corner_factors(pr.ax, pr.ay, c, wx, wy);
            go = __builtin_fma((double)wx * (double)wy, (double)da[c], go);
            const int64_t q = V.pixel_offset + (int64_t)(y0 + (c >> 1)) * V.W + (x0 + (c & 1));
            float g[FM];
            f32_row<FM, DYN>(g_img, q, Fd, g);
#pragma unroll
            for (int f = 0; f < FM; ++f) gf[f] = __builtin_fma((double)ta[c], (double)g[f], gf[f]);
        }
    }
    float out[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) out[f] = (float)gf[f];
    f32_store<FM, DYN>(grad_feat, vp, Fd, out);
    grad_opa[vp] = (float)go;
}

// ------------------------------------------------ view -> point gradients
template <int FM, bool DYN>
__global__ __launch_bounds__(256) void k_sum_view_grads(
    const GpuView* __restrict__ views, int n_views, int64_t n_points, int Fd,
    const float* __restrict__ vg_feat, const float* __restrict__ vg_opa, float* __restrict__ g_feat,
    float* __restrict__ g_opa) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_points) return;
    float gf[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) gf[f] = 0.0f;
    float go = 0.0f;
    for (int v = 0; v < n_views; ++v) {
        const GpuView& V = views[v];
        if (p < V.point_offset || p >= V.point_offset + V.point_count) continue;
        const int64_t vp = V.vpoint_offset + (p - V.point_offset);
        float g[FM];
        f32_row<FM, DYN>(vg_feat, vp, Fd, g);
#pragma unroll
        for (int f = 0; f < FM; ++f) gf[f] += g[f];
        go += vg_opa[vp];
    }
    f32_store<FM, DYN>(g_feat, p, Fd, gf);
    g_opa[p] = go;
}

// ------------------------------------------------------------- dispatch
template <typename FT, int FM, bool DYN, int WX>
static void blend_fwd_t(const GpuView* views, int n_views, int64_t n_tiles, const uint2* range,
                        const uint32_t* ids, const PointRec* rec, const void* feat, int Fd, float tau,
                        float* image, float* t_final, PixelState* state, float* t_before, hipStream_t s) {
    hipLaunchKernelGGL((k_blend_fwd<FT, FM, DYN, WX>), dim3((unsigned)n_tiles), dim3(256), 0, s, views,
                       n_views, range, ids, rec, reinterpret_cast<const FT*>(feat), Fd, tau, image,
                       t_final, state, t_before);
}

template <typename FT, int FM, bool DYN, int WX>
static void blend_bwd_t(const GpuView* views, int n_views, int64_t n_tiles, const uint2* range,
                        const uint32_t* ids, const PointRec* rec, const void* feat, int Fd,
                        const PixelState* state, const float* g_img, const float* g_t, float* t_before,
                        int rebuild_t, float2* frec, hipStream_t s) {
    hipLaunchKernelGGL((k_blend_bwd<FT, FM, DYN, WX>), dim3((unsigned)n_tiles), dim3(256), 0, s, views,
                       n_views, range, ids, rec, reinterpret_cast<const FT*>(feat), Fd, state, g_img,
                       g_t, t_before, rebuild_t, frec);
}

// Calls body.template operator()<FM, DYN>() for the compiled feature widths.
template <typename Body>
static bool dispatch_f(int F, Body&& body) {
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

template <typename Body>
static void dispatch_wx(int wave_x, Body&& body) {
    switch (wave_x) {
        case 16: body.template operator()<16>(); break;
        case 4: body.template operator()<4>(); break;
        default: body.template operator()<8>(); break;
    }
}

void launch_blend_fwd(int F, int feat_dtype, int wave_x, const GpuView* views, int n_views,
                      int64_t n_tiles, const uint2* range, const uint32_t* ids, const PointRec* rec,
                      const void* feat, float tau, float* image, float* t_final, PixelState* state,
                      float* t_before, hipStream_t s) {
    if (n_tiles == 0) return;
    dispatch_f(F, [&]<int FM, bool DYN>() {
        dispatch_wx(wave_x, [&]<int WX>() {
            if (feat_dtype == 1)
                blend_fwd_t<__hip_bfloat16, FM, DYN, WX>(views, n_views, n_tiles, range, ids, rec, feat, F,
                                                         tau, image, t_final, state, t_before, s);
            else
                blend_fwd_t<float, FM, DYN, WX>(views, n_views, n_tiles, range, ids, rec, feat, F, tau,
                                                image, t_final, state, t_before, s);
        });
    });
}

void launch_blend_bwd(int F, int feat_dtype, int wave_x, const GpuView* views, int n_views,
                      int64_t n_tiles, const uint2* range, const uint32_t* ids, const PointRec* rec,
                      const void* feat, const PixelState* state, const float* g_img,
                      const float* g_t, float* t_before, int rebuild_t, float2* frec, hipStream_t s) {
    if (n_tiles == 0) return;
    dispatch_f(F, [&]<int FM, bool DYN>() {
        dispatch_wx(wave_x, [&]<int WX>() {
            if (feat_dtype == 1)
                blend_bwd_t<__hip_bfloat16, FM, DYN, WX>(views, n_views, n_tiles, range, ids, rec, feat, F,
                                                         state, g_img, g_t, t_before, rebuild_t, frec, s);
            else
                blend_bwd_t<float, FM, DYN, WX>(views, n_views, n_tiles, range, ids, rec, feat, F, state,
                                                g_img, g_t, t_before, rebuild_t, frec, s);
        });
    });
}

void launch_point_reduce(int F, const GpuView* views, int n_views, int64_t n_vp,
                         const PointRec* rec, const float2* frec, const float* g_img,
                         float* grad_feat, float* grad_opa, hipStream_t s) {
    if (n_vp == 0) return;
    const unsigned blocks = (unsigned)((n_vp + 255) / 256);
    dispatch_f(F, [&]<int FM, bool DYN>() {
        hipLaunchKernelGGL((k_point_reduce<FM, DYN>), dim3(blocks), dim3(256), 0, s, views, n_views, n_vp,
                           rec, frec, g_img, F, grad_feat, grad_opa);
    });
}

void launch_sum_view_grads(const GpuView* views, int n_views, int64_t n_points, int F,
                           const float* vg_feat, const float* vg_opa, float* g_feat, float* g_opa,
                           hipStream_t s) {
    if (n_points == 0) return;
    const unsigned blocks = (unsigned)((n_points + 255) / 256);
    dispatch_f(F, [&]<int FM, bool DYN>() {
        hipLaunchKernelGGL((k_sum_view_grads<FM, DYN>), dim3(blocks), dim3(256), 0, s, views, n_views,
                           n_points, F, vg_feat, vg_opa, g_feat, g_opa);
    });
}

}  // namespace inpc
