// Forward blend (Eq. 1 with early termination; the BlendSortedSplats step
// of Algorithm 1) for gfx950.
//
// L lanes share one pixel: in each step the L lanes gather L consecutive
// splats of the pixel's depth-sorted list at once (independent loads), form
// the transmittance in front of each with a prefix product of (1 - alpha)
// across the group, and accumulate their own share of the colour; the
// shares are summed across the group once at the end.  This keeps L
// gathers in flight per pixel and divides the longest list of a wave by L.
#include "blend_common.h"

namespace inpc {

template <typename FT, int FM, bool DYN, int WXP, int L>
__global__ __launch_bounds__(256) void k_blend_fwd(
    const GpuView* __restrict__ views, int n_views, const uint2* __restrict__ range,
    const uint32_t* __restrict__ ids, const PointRec* __restrict__ rec, const FT* __restrict__ feat,
    int Fd, float tau, float* __restrict__ image, float* __restrict__ t_final,
    PixelState* __restrict__ state, float* __restrict__ t_before, float* __restrict__ splat_weight) {
    const TileCoord tc = tile_pixel<WXP, L>(views, n_views);
    if (!tc.inside) return;
    const int sub = __lane_id() % L;
    const int64_t pbase = tc.V->attr_offset - tc.V->vpoint_offset;
    const uint2 r = range[tc.q];
    float C[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) C[f] = 0.0f;
    float T = 1.0f;
    uint32_t nb = 0;
    for (uint32_t base = r.x; base < r.y; base += L) {
        const uint32_t i = base + sub;
        const bool valid = i < r.y;
        float cf[FM];
        float alpha = 0.0f, om = 1.0f;
        uint32_t id = 0;
        if (valid) {
            id = ids[i];
            const uint32_t vp = id >> 2;
            const PointRec pr = rec[vp];
            feat_row<FT, FM, DYN>(feat, pbase + vp, Fd, cf);
            float wx, wy;
            corner_factors(pr.ax, pr.ay, (int)(id & 3u), wx, wy);
            splat_alpha(pr.opa, wx, wy, alpha, om);
        } else {
#pragma unroll
            for (int f = 0; f < FM; ++f) cf[f] = 0.0f;
        }
        const GroupStep g = group_step<L>(T, om, valid, base == r.x && sub == 0, tau, sub);
        if (g.blended) {
            const float ta = g.tb * alpha;
#pragma unroll
            for (int f = 0; f < FM; ++f) C[f] = __builtin_fmaf(ta, cf[f], C[f]);
            if (t_before) t_before[i] = g.tb;
            if (splat_weight) splat_weight[id] = ta;
            ++nb;
        }
        T = g.t_next;
        if (g.done) break;
    }
#pragma unroll
    for (int m = L / 2; m >= 1; m >>= 1) {
#pragma unroll
        for (int f = 0; f < FM; ++f) C[f] += __shfl_xor(C[f], m, L);
        nb += __shfl_xor(nb, m, L);
    }
    if (sub == 0) {
        f32_store<FM, DYN>(image, tc.q, Fd, C);
        t_final[tc.q] = T;
        PixelState st;
        st.n_blended = nb;
        st.pad0 = st.pad1 = st.pad2 = 0;
        state[tc.q] = st;
    }
}

template <typename FT, int FM, bool DYN, int WXP, int L>
static void blend_fwd_t(const GpuView* views, int n_views, int64_t n_tiles, const uint2* range,
                        const uint32_t* ids, const PointRec* rec, const void* feat, int Fd, float tau,
                        float* image, float* t_final, PixelState* state, float* t_before,
                        float* splat_weight, hipStream_t s) {
    hipLaunchKernelGGL((k_blend_fwd<FT, FM, DYN, WXP, L>), dim3((unsigned)n_tiles), dim3(256), 0, s, views,
                       n_views, range, ids, rec, reinterpret_cast<const FT*>(feat), Fd, tau, image,
                       t_final, state, t_before, splat_weight);
}

void launch_blend_fwd(int F, int feat_dtype, int shape, const GpuView* views, int n_views,
                      int64_t n_tiles, const uint2* range, const uint32_t* ids, const PointRec* rec,
                      const void* feat, float tau, float* image, float* t_final, PixelState* state,
                      float* t_before, float* splat_weight, hipStream_t s) {
    if (n_tiles == 0) return;
    dispatch_f(F, [&]<int FM, bool DYN>() {
        dispatch_shape(shape, [&]<int WXP, int L>() {
            if (feat_dtype == 1)
                blend_fwd_t<__hip_bfloat16, FM, DYN, WXP, L>(views, n_views, n_tiles, range, ids, rec, feat,
                                                             F, tau, image, t_final, state, t_before,
                                                             splat_weight, s);
            else
                blend_fwd_t<float, FM, DYN, WXP, L>(views, n_views, n_tiles, range, ids, rec, feat, F, tau,
                                                    image, t_final, state, t_before, splat_weight, s);
        });
    });
}

}  // namespace inpc
