// Deterministic per-point gradient reduction (Appendix A.6: a point's
// gradient combines its splat gradients weighted by the bilinear weights)
// and the fold of per-view-point gradients onto shared points, for gfx950.
#include "blend_common.h"

namespace inpc {

// --------------------------------------------------- per-point reduction
// grad_opa[vp] = sum_c w_c dL/dalpha_c, grad_feat[vp] = sum_c T_c alpha_c g_{pixel(c)}
// and, if requested, the blend weight b[vp] = sum_c w_c T_c alpha_c
// over the existing corners c = 0..3 in ascending order; the per-splat
// records of a point are contiguous (ids 4vp .. 4vp+3), so this is a
// segmented reduction over the id-ordered splat records.  Non-blended
// splats hold zeros (the record array is cleared before the backward blend).
template <int FM, bool DYN>
__global__ __launch_bounds__(256) void k_point_reduce(
    const GpuView* __restrict__ views, int n_views, int64_t n_vp, const PointRec* __restrict__ rec,
    const float2* __restrict__ frec, const float* __restrict__ g_img, int Fd,
    float* __restrict__ grad_feat, float* __restrict__ grad_opa, float* __restrict__ blend_weight) {
    const int64_t vp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // The point's record, its four splat records (zero where nothing was
    // blended) and its view's placement are read together, and for narrow
    // rows the gradient rows of all corners are in flight before the first
    // one is used: each point waits on two memory latencies, not one per
    // read.  No load sits under a branch (a point without splats reads its
    // view's first pixel row and ignores it), so the compiler cannot sink the
    // record loads behind the wait for the point record.  The block's view
    // is looked up once (uniform); a block across two views searches per
    // thread.
    auto vstart = [](const GpuView& g) { return g.vpoint_offset; };
    const int64_t vpb = (int64_t)blockIdx.x * blockDim.x;
    const int v0 = n_views == 1 ? 0 : find_view(views, n_views, vpb, vstart);
    const bool one_view = n_views == 1 || vpb + (int64_t)blockDim.x <= views[v0].vpoint_offset + views[v0].point_count;
    if (vp >= n_vp) return;
    int64_t pix0, W;
    if (one_view) {
        pix0 = views[v0].pixel_offset;
        W = views[v0].W;
    } else {
        const int v = find_view(views, n_views, vp, vstart);
        pix0 = views[v].pixel_offset;
        W = views[v].W;
    }
    const PointRec pr = rec[vp];
    const float4 r01 = reinterpret_cast<const float4*>(frec)[2 * vp];
    const float4 r23 = reinterpret_cast<const float4*>(frec)[2 * vp + 1];
    const uint32_t mask = anc_mask(pr.anc);
    const float da[4] = {r01.x, r01.z, r23.x, r23.z};
    const float ta[4] = {r01.y, r01.w, r23.y, r23.w};
    // pixel of each corner; a missing corner (off the image or of zero
    // weight) reads the row of the first present one
    const int x0 = anc_x0(pr.anc), y0 = anc_y0(pr.anc);
    const int cf = mask != 0u ? __builtin_ctz(mask) : 0;
    int64_t q[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int cc = ((mask >> c) & 1u) ? c : cf;
        q[c] = mask != 0u ? pix0 + (int64_t)(y0 + (cc >> 1)) * W + (x0 + (cc & 1)) : pix0;
    }
    // float64 accumulators: the (at most four) corner terms often cancel.
    double gf[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) gf[f] = 0.0;
    double go = 0.0, bw = 0.0;
    // the terms of corner c, kept only if the corner exists (a select, so
    // the result equals skipping the corner bit for bit, and the row's loads
    // have a use on every path)
    auto corner_terms = [&](int c, const float (&g)[FM]) {
        const bool on = (mask >> c) & 1u;
        float wx, wy;
        corner_factors(pr.ax, pr.ay, c, wx, wy);
        const double go2 = __builtin_fma((double)wx * (double)wy, (double)da[c], go);
        const double bw2 = __builtin_fma((double)wx * (double)wy, (double)ta[c], bw);
        go = on ? go2 : go;
        bw = on ? bw2 : bw;
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            const double t = __builtin_fma((double)ta[c], (double)g[f], gf[f]);
            gf[f] = on ? t : gf[f];
        }
    };
    if constexpr (FM <= 16) {
        float g[4][FM];
#pragma unroll
        for (int c = 0; c < 4; ++c) f32_row<FM, DYN>(g_img, q[c], Fd, g[c]);
#pragma unroll
        for (int c = 0; c < 4; ++c) corner_terms(c, g[c]);
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!((mask >> c) & 1u)) continue;
            float g[FM];
            f32_row<FM, DYN>(g_img, q[c], Fd, g);
            corner_terms(c, g);
        }
    }
    float out[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) out[f] = (float)gf[f];
    f32_store<FM, DYN>(grad_feat, vp, Fd, out);
    grad_opa[vp] = (float)go;
    if (blend_weight) blend_weight[vp] = (float)bw;
}

// The same reduction with S = FM / 4 lanes per point, lane s owning
// features 4s .. 4s+3: one wave load then covers the 64-byte gradient rows of
// 16 points (whole rows, 16 lines) instead of one 16-byte piece of each of 64
// rows, and the gradient rows are stored as one contiguous run per wave.
// Every lane forms the point's terms in the same order as above, so the
// results are bit-identical; lane 0 of the point writes the scalars.
template <int FM>
__global__ __launch_bounds__(256) void k_point_reduce_q(
    const GpuView* __restrict__ views, int n_views, int64_t n_vp, const PointRec* __restrict__ rec,
    const float2* __restrict__ frec, const float* __restrict__ g_img, float* __restrict__ grad_feat,
    float* __restrict__ grad_opa, float* __restrict__ blend_weight) {
    constexpr int S = FM / 4;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t vp = t / S;
    const int sub = (int)(t % S);
    // the block's view once (uniform); a block across two views searches per thread
    auto vstart = [](const GpuView& g) { return g.vpoint_offset; };
    const int64_t vpb = (int64_t)blockIdx.x * (256 / S);
    const int v0 = n_views == 1 ? 0 : find_view(views, n_views, vpb, vstart);
    const bool one_view = n_views == 1 || vpb + 256 / S <= views[v0].vpoint_offset + views[v0].point_count;
    if (vp >= n_vp) return;
    int64_t pix0, W;
    if (one_view) {
        pix0 = views[v0].pixel_offset;
        W = views[v0].W;
    } else {
        const int v = find_view(views, n_views, vp, vstart);
        pix0 = views[v].pixel_offset;
        W = views[v].W;
    }
    const PointRec pr = rec[vp];
    const float4 r01 = reinterpret_cast<const float4*>(frec)[2 * vp];
    const float4 r23 = reinterpret_cast<const float4*>(frec)[2 * vp + 1];
    const uint32_t mask = anc_mask(pr.anc);
    const float da[4] = {r01.x, r01.z, r23.x, r23.z};
    const float ta[4] = {r01.y, r01.w, r23.y, r23.w};
    const int x0 = anc_x0(pr.anc), y0 = anc_y0(pr.anc);
    const int cf = mask != 0u ? __builtin_ctz(mask) : 0;
    float4 g[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int cc = ((mask >> c) & 1u) ? c : cf;
        const int64_t q = mask != 0u ? pix0 + (int64_t)(y0 + (cc >> 1)) * W + (x0 + (cc & 1)) : pix0;
        g[c] = reinterpret_cast<const float4*>(g_img + q * FM)[sub];
    }
    double gf[4] = {0.0, 0.0, 0.0, 0.0};
    double go = 0.0, bw = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const bool on = (mask >> c) & 1u;
        float wx, wy;
        corner_factors(pr.ax, pr.ay, c, wx, wy);
        const double go2 = __builtin_fma((double)wx * (double)wy, (double)da[c], go);
        const double bw2 = __builtin_fma((double)wx * (double)wy, (double)ta[c], bw);
        go = on ? go2 : go;
        bw = on ? bw2 : bw;
        const float gc[4] = {g[c].x, g[c].y, g[c].z, g[c].w};
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const double x = __builtin_fma((double)ta[c], (double)gc[f], gf[f]);
            gf[f] = on ? x : gf[f];
        }
    }
    reinterpret_cast<float4*>(grad_feat + vp * FM)[sub] =
        make_float4((float)gf[0], (float)gf[1], (float)gf[2], (float)gf[3]);
    if (sub == 0) {
        grad_opa[vp] = (float)go;
        if (blend_weight) blend_weight[vp] = (float)bw;
    }
}

// ------------------------------------------------ per-point blend weight
// b[vp] = sum over the existing corners c (ascending) of w_c * T_c alpha_c:
// the splat blend weights of Eq. 1 combined with the bilinear weights as
// factors (Appendix A.6), the per-point quantity the probability updates of
// Section 3.1 consume.  Splats that were not blended hold zeros (the
// per-splat array is cleared before the forward blend).
__global__ __launch_bounds__(256) void k_blend_weight(int64_t n_vp, const PointRec* __restrict__ rec,
                                                      const float* __restrict__ splat_weight,
                                                      float* __restrict__ out) {
    const int64_t vp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (vp >= n_vp) return;
    const PointRec pr = rec[vp];
    const uint32_t mask = anc_mask(pr.anc);
    double b = 0.0;
    if (mask != 0u) {
        const float4 sw = reinterpret_cast<const float4*>(splat_weight)[vp];
        const float s4[4] = {sw.x, sw.y, sw.z, sw.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!((mask >> c) & 1u)) continue;
            float wx, wy;
            corner_factors(pr.ax, pr.ay, c, wx, wy);
            b = __builtin_fma((double)wx * (double)wy, (double)s4[c], b);
        }
    }
    out[vp] = (float)b;
}

void launch_blend_weight(int64_t n_vp, const PointRec* rec, const float* splat_weight, float* out,
                         hipStream_t s) {
    if (n_vp == 0) return;
    hipLaunchKernelGGL(k_blend_weight, dim3((unsigned)((n_vp + 255) / 256)), dim3(256), 0, s, n_vp, rec,
                       splat_weight, out);
}

// ------------------------------------------------ multisample average
// out[i] = (sum_k in[k * plane + i]) / K with the sum in float64 in ascending
// k and one correctly rounded division: the per-pixel average of K feature
// images of one view (Section 3.2, inference with several sampled clouds).
template <bool VEC>
__global__ __launch_bounds__(256) void k_mean_planes(const float* __restrict__ in, int K, int64_t plane,
                                                     float* __restrict__ out) {
    const double dk = (double)K;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if constexpr (VEC) {
        const int64_t n4 = plane / 4;
        const float4* src = reinterpret_cast<const float4*>(in);
        float4* dst = reinterpret_cast<float4*>(out);
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
            double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
            for (int k = 0; k < K; ++k) {
                const float4 x = src[(int64_t)k * n4 + i];
                a += (double)x.x;
                b += (double)x.y;
                c += (double)x.z;
                d += (double)x.w;
            }
            dst[i] = make_float4((float)(a / dk), (float)(b / dk), (float)(c / dk), (float)(d / dk));
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < plane; i += stride) {
            double a = 0.0;
            for (int k = 0; k < K; ++k) a += (double)in[(int64_t)k * plane + i];
            out[i] = (float)(a / dk);
        }
    }
}

void launch_mean_planes(const float* in, int K, int64_t plane, float* out, hipStream_t s) {
    if (plane == 0) return;
    const bool vec = (plane % 4) == 0 && (reinterpret_cast<uintptr_t>(in) % 16) == 0 &&
                     (reinterpret_cast<uintptr_t>(out) % 16) == 0;
    const int64_t items = vec ? plane / 4 : plane;
    int64_t blocks = (items + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (vec)
        hipLaunchKernelGGL(k_mean_planes<true>, dim3((unsigned)blocks), dim3(256), 0, s, in, K, plane, out);
    else
        hipLaunchKernelGGL(k_mean_planes<false>, dim3((unsigned)blocks), dim3(256), 0, s, in, K, plane, out);
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
                         float* grad_feat, float* grad_opa, float* blend_weight, hipStream_t s) {
    if (n_vp == 0) return;
    // rows of 8, 16 or 32 float32 (16-byte aligned): F / 4 lanes per point,
    // while the grid stays below 2^31 work items
    if ((F == 8 || F == 16 || F == 32) && n_vp <= ((int64_t)1 << 31) / (F / 4)) {
        const int64_t threads = n_vp * (F / 4);
        const unsigned qblocks = (unsigned)((threads + 255) / 256);
        auto q = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3(qblocks), dim3(256), 0, s, views, n_views, n_vp, rec, frec, g_img,
                               grad_feat, grad_opa, blend_weight);
        };
        if (F == 8) q(k_point_reduce_q<8>);
        else if (F == 16) q(k_point_reduce_q<16>);
        else q(k_point_reduce_q<32>);
        return;
    }
    const unsigned blocks = (unsigned)((n_vp + 255) / 256);
    dispatch_f(F, [&]<int FM, bool DYN>() {
        hipLaunchKernelGGL((k_point_reduce<FM, DYN>), dim3(blocks), dim3(256), 0, s, views, n_views, n_vp,
                           rec, frec, g_img, F, grad_feat, grad_opa, blend_weight);
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
