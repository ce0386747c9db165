// Deterministic per-point gradient reduction (Appendix A.6: a point's
// gradient combines its splat gradients weighted by the bilinear weights)
// and the fold of per-view-point gradients onto shared points, for gfx950.
#include "blend_common.h"

namespace inpc {

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
