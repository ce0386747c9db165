// Backward of the blend (Appendix A.6: per-splat gradients in the order of
// the forward pass) for gfx950.
//
// For the blended splats k = 0 .. n-1 of a pixel, with
// Y_k = alpha_k (g.c_k) + (1 - alpha_k) Y_{k+1} and Y_n = g_T,
//   dL/dalpha_k = T_k ((g.c_k) - Y_{k+1}),   dL/dc_k = T_k alpha_k g.
// The list is walked from its end in groups of L splats held by the L lanes
// of the pixel; inside a group Y_{k+1} comes from a suffix scan of the affine
// maps Y -> alpha_k (g.c_k) + (1 - alpha_k) Y.  T_k is the forward's own
// float32 value (stored per blended splat by the forward, or rebuilt here by
// the forward's group recurrence).  The scalar chain runs in float64
// registers: dL/dalpha is a difference of two nearly equal sums for many
// splats.  Each splat's record (dL/dalpha_k, T_k alpha_k) is written at its
// splat id 4p + corner.
#include "blend_common.h"

namespace inpc {

template <typename FT, int FM, bool DYN, int WXP, int L>
__global__ __launch_bounds__(256) void k_blend_bwd(
    const GpuView* __restrict__ views, int n_views, const uint2* __restrict__ range,
    const uint32_t* __restrict__ ids, const PointRec* __restrict__ rec, const FT* __restrict__ feat,
    int Fd, float tau, const PixelState* __restrict__ state, const float* __restrict__ g_img,
    const float* __restrict__ g_t, float* __restrict__ t_before, int rebuild_t,
    float2* __restrict__ frec) {
    const TileCoord tc = tile_pixel<WXP, L>(views, n_views);
    if (!tc.inside) return;
    const int sub = __lane_id() % L;
    const uint32_t n = state[tc.q].n_blended;
    if (n == 0) return;
    const int64_t pbase = tc.V->attr_offset - tc.V->vpoint_offset;
    const uint32_t start = range[tc.q].x;
    if (rebuild_t) {
        // Same group recurrence as the forward over the blended prefix.
        float T = 1.0f;
        for (uint32_t base = start; base < start + n; base += L) {
            const uint32_t i = base + sub;
            const bool valid = i < start + n;
            float alpha = 0.0f, om = 1.0f;
            if (valid) {
                const uint32_t id = ids[i];
                const PointRec pr = rec[id >> 2];
                float wx, wy;
                corner_factors(pr.ax, pr.ay, (int)(id & 3u), wx, wy);
                splat_alpha(pr.opa, wx, wy, alpha, om);
            }
            const GroupStep g = group_step<L>(T, om, valid, base == start && sub == 0, tau, sub);
            if (valid) t_before[i] = g.tb;
            T = g.t_next;
        }
    }
    float g[FM];
    f32_row<FM, DYN>(g_img, tc.q, Fd, g);
    double Y = g_t ? (double)g_t[tc.q] : 0.0;
    const int groups = (int)((n + L - 1) / L);
    for (int gi = groups - 1; gi >= 0; --gi) {
        const uint32_t k = (uint32_t)gi * L + sub;
        const bool valid = k < n;
        double A = 0.0, B = 1.0, alpha = 0.0, gc = 0.0, Tk = 0.0;
        uint32_t id = 0;
        if (valid) {
            id = ids[start + k];
            const uint32_t vp = id >> 2;
            const PointRec pr = rec[vp];
            float cf[FM];
            feat_row<FT, FM, DYN>(feat, pbase + vp, Fd, cf);
            float wx, wy;
            corner_factors(pr.ax, pr.ay, (int)(id & 3u), wx, wy);
            alpha = (double)pr.opa * ((double)wx * (double)wy);
#pragma unroll
            for (int f = 0; f < FM; ++f) gc = __builtin_fma((double)g[f], (double)cf[f], gc);
            Tk = (double)t_before[start + k];
            A = alpha * gc;
            B = 1.0 - alpha;
        }
        // inclusive suffix composition of the maps of lanes sub .. L-1
#pragma unroll
        for (int d = 1; d < L; d <<= 1) {
            const double A2 = __shfl_down(A, d, L);
            const double B2 = __shfl_down(B, d, L);
            if (sub + d < L) {
                A = __builtin_fma(B, A2, A);
                B = B * B2;
            }
        }
        double Ae = __shfl_down(A, 1, L), Be = __shfl_down(B, 1, L);
        if (sub == L - 1) {
            Ae = 0.0;
            Be = 1.0;
        }
        const double y_next = __builtin_fma(Be, Y, Ae);
        if (valid) frec[id] = make_float2((float)(Tk * (gc - y_next)), (float)(Tk * alpha));
        Y = __builtin_fma(__shfl(B, 0, L), Y, __shfl(A, 0, L));
    }
}

template <typename FT, int FM, bool DYN, int WXP, int L>
static void blend_bwd_t(const GpuView* views, int n_views, int64_t n_tiles, const uint2* range,
                        const uint32_t* ids, const PointRec* rec, const void* feat, int Fd, float tau,
                        const PixelState* state, const float* g_img, const float* g_t, float* t_before,
                        int rebuild_t, float2* frec, hipStream_t s) {
    hipLaunchKernelGGL((k_blend_bwd<FT, FM, DYN, WXP, L>), dim3((unsigned)n_tiles), dim3(256), 0, s, views,
                       n_views, range, ids, rec, reinterpret_cast<const FT*>(feat), Fd, tau, state, g_img,
                       g_t, t_before, rebuild_t, frec);
}

void launch_blend_bwd(int F, int feat_dtype, int shape, const GpuView* views, int n_views,
                      int64_t n_tiles, const uint2* range, const uint32_t* ids, const PointRec* rec,
                      const void* feat, float tau, const PixelState* state, const float* g_img,
                      const float* g_t, float* t_before, int rebuild_t, float2* frec, hipStream_t s) {
    if (n_tiles == 0) return;
    dispatch_f(F, [&]<int FM, bool DYN>() {
        dispatch_shape(shape, [&]<int WXP, int L>() {
            if (feat_dtype == 1)
                blend_bwd_t<__hip_bfloat16, FM, DYN, WXP, L>(views, n_views, n_tiles, range, ids, rec, feat,
                                                             F, tau, state, g_img, g_t, t_before, rebuild_t,
                                                             frec, s);
            else
                blend_bwd_t<float, FM, DYN, WXP, L>(views, n_views, n_tiles, range, ids, rec, feat, F, tau,
                                                    state, g_img, g_t, t_before, rebuild_t, frec, s);
        });
    });
}

}  // namespace inpc
