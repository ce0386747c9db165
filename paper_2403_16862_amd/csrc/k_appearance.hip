// Per-point appearance step (Section 3.3) for gfx950: the opacity
// activation alpha_h = 1 - exp(-exp(x)) and the degree-2 spherical-harmonics
// evaluation that turns 36 coefficients into a 4-D view-dependent feature,
// plus its backward.  Raw rows are [1 + 36] floats: the opacity logit, then
// coefficient (basis j, channel c) at 1 + 4 j + c.
//
// Rows of 37 floats are not 16-byte aligned individually, but the rows of a
// block of 256 points are one contiguous run: a block stages them through
// LDS with coalesced 16-byte accesses (dwords where the run is not aligned)
// and each thread then reads its own row at an odd LDS stride (37 words: no
// bank conflicts).
#include "internal.h"

namespace inpc {

constexpr int kRawW = 37;
constexpr int kApBlock = 256;

// Block copy of ``n`` floats between global memory and LDS: 16-byte accesses
// when both sides allow them, dwords for the rest.
template <bool TO_LDS>
__device__ __forceinline__ void stage_rows(float* __restrict__ lds, float* __restrict__ glob, int n) {
    int done = 0;
    if ((reinterpret_cast<uintptr_t>(glob) & 15u) == 0) {
        const int n4 = n >> 2;
        float4* l4 = reinterpret_cast<float4*>(lds);
        float4* g4 = reinterpret_cast<float4*>(glob);
        for (int e = threadIdx.x; e < n4; e += kApBlock) {
            if constexpr (TO_LDS) l4[e] = g4[e];
            else g4[e] = l4[e];
        }
        done = n4 << 2;
    }
    for (int e = done + threadIdx.x; e < n; e += kApBlock) {
        if constexpr (TO_LDS) lds[e] = glob[e];
        else glob[e] = lds[e];
    }
}

// Real SH basis of degree <= 2 at the unit direction (x, y, z), in the order
// (0,0), (1,-1), (1,0), (1,1), (2,-2), (2,-1), (2,0), (2,1), (2,2); the real
// functions are sqrt(2) Re / Im of the complex ones with the Condon-Shortley
// phase (the usual graphics convention).  Constants: 1/(2 sqrt(pi)),
// sqrt(3/(4 pi)), sqrt(15/(4 pi)), sqrt(5/(16 pi)), sqrt(15/(16 pi)).
__device__ __forceinline__ void sh2_basis(float x, float y, float z, float (&Y)[9]) {
    const float k0 = 0.28209479177387814f, k1 = 0.48860251190291992f, k2 = 1.0925484305920792f,
                k20 = 0.31539156525252005f, k22 = 0.54627421529603959f;
    Y[0] = k0;
    Y[1] = -k1 * y;
    Y[2] = k1 * z;
    Y[3] = -k1 * x;
    Y[4] = k2 * (x * y);
    Y[5] = -k2 * (y * z);
    Y[6] = k20 * (3.0f * (z * z) - 1.0f);
    Y[7] = -k2 * (x * z);
    Y[8] = k22 * (x * x - y * y);
}

// Unit vector from the camera centre o = -R^T t to the point; the zero
// vector for a point at the centre (such points are never rendered, and the
// zero direction keeps their gradients finite).
__device__ __forceinline__ void view_dir(const GpuView& V, float px, float py, float pz, float& dx,
                                         float& dy, float& dz) {
    const float ox = -(V.R[0] * V.t[0] + V.R[3] * V.t[1] + V.R[6] * V.t[2]);
    const float oy = -(V.R[1] * V.t[0] + V.R[4] * V.t[1] + V.R[7] * V.t[2]);
    const float oz = -(V.R[2] * V.t[0] + V.R[5] * V.t[1] + V.R[8] * V.t[2]);
    dx = px - ox;
    dy = py - oy;
    dz = pz - oz;
    const float n2 = dx * dx + dy * dy + dz * dz;
    const float inv = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
    dx *= inv;
    dy *= inv;
    dz *= inv;
}

template <bool BF16>
__global__ __launch_bounds__(kApBlock) void k_appearance_fwd(const float* __restrict__ xyz,
                                                             const float* __restrict__ raw,
                                                             const GpuView* __restrict__ views, int n_views,
                                                             int64_t n_vp, float* __restrict__ opa_out,
                                                             void* __restrict__ feat_out) {
    __shared__ __align__(16) float s_raw[kApBlock * kRawW];
    const int64_t vp0 = (int64_t)blockIdx.x * kApBlock;
    const int rows = (int)((n_vp - vp0) < kApBlock ? (n_vp - vp0) : kApBlock);
    auto vstart = [](const GpuView& g) { return g.vpoint_offset; };
    const int v0 = n_views == 1 ? 0 : find_view(views, n_views, vp0, vstart);
    const GpuView& V0 = views[v0];
    // Fast path: all rows of the block belong to one view, so their raw rows
    // are contiguous in memory.
    const bool one_view = vp0 + rows <= V0.vpoint_offset + V0.point_count;
    if (one_view)
        stage_rows<true>(s_raw, const_cast<float*>(raw) + (V0.point_offset + (vp0 - V0.vpoint_offset)) * kRawW,
                         rows * kRawW);
    __syncthreads();
    const int64_t vp = vp0 + threadIdx.x;
    if (vp >= n_vp) return;
    const int v = one_view ? v0 : find_view(views, n_views, vp, vstart);
    const GpuView& V = views[v];
    const int64_t p = V.point_offset + (vp - V.vpoint_offset);
    float r[kRawW];
    if (one_view) {
#pragma unroll
        for (int j = 0; j < kRawW; ++j) r[j] = s_raw[threadIdx.x * kRawW + j];
    } else {
#pragma unroll
        for (int j = 0; j < kRawW; ++j) r[j] = raw[p * kRawW + j];
    }
    float dx, dy, dz;
    view_dir(V, xyz[3 * p], xyz[3 * p + 1], xyz[3 * p + 2], dx, dy, dz);
    float Y[9];
    sh2_basis(dx, dy, dz, Y);
    float f[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float a = 0.0f;
#pragma unroll
        for (int j = 0; j < 9; ++j) a = __builtin_fmaf(Y[j], r[1 + 4 * j + c], a);
        f[c] = a;
    }
    // 1 - exp(-exp(x)) = -expm1(-exp(x)), evaluated in float64 and rounded
    // once, so small opacities keep their relative precision.
    opa_out[vp] = (float)(-expm1(-exp((double)r[0])));
    if constexpr (BF16) {
        uint2 w;
        w.x = f32_to_bf16_bits(f[0]) | (f32_to_bf16_bits(f[1]) << 16);
        w.y = f32_to_bf16_bits(f[2]) | (f32_to_bf16_bits(f[3]) << 16);
        reinterpret_cast<uint2*>(feat_out)[vp] = w;
    } else {
        reinterpret_cast<float4*>(feat_out)[vp] = make_float4(f[0], f[1], f[2], f[3]);
    }
}

// grad_raw[p] = sum over the views containing p, in view order, of
// (g_opa[vp] * d alpha_h / dx, Y_j(d_v) g_feat[vp][c]); float64 sums.
__global__ __launch_bounds__(kApBlock) void k_appearance_bwd(const float* __restrict__ xyz,
                                                             const float* __restrict__ raw,
                                                             const GpuView* __restrict__ views, int n_views,
                                                             int64_t n_points, const float* __restrict__ g_opa,
                                                             const float* __restrict__ g_feat,
                                                             float* __restrict__ grad_raw) {
    __shared__ __align__(16) float s_out[kApBlock * kRawW];
    const int64_t p0 = (int64_t)blockIdx.x * kApBlock;
    const int rows = (int)((n_points - p0) < kApBlock ? (n_points - p0) : kApBlock);
    const int64_t p = p0 + threadIdx.x;
    if (p < n_points) {
        double acc[kRawW];
#pragma unroll
        for (int j = 0; j < kRawW; ++j) acc[j] = 0.0;
        const float px = xyz[3 * p], py = xyz[3 * p + 1], pz = xyz[3 * p + 2];
        const double x0 = (double)raw[p * kRawW];
        const double dact = exp(x0 - exp(x0));
        for (int v = 0; v < n_views; ++v) {
            const GpuView& V = views[v];
            if (p < V.point_offset || p >= V.point_offset + V.point_count) continue;
            const int64_t vp = V.vpoint_offset + (p - V.point_offset);
            const float4 g = reinterpret_cast<const float4*>(g_feat)[vp];
            acc[0] += (double)g_opa[vp] * dact;
            float dx, dy, dz;
            view_dir(V, px, py, pz, dx, dy, dz);
            float Y[9];
            sh2_basis(dx, dy, dz, Y);
            const float gc[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
            for (int j = 0; j < 9; ++j)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[1 + 4 * j + c] += (double)Y[j] * (double)gc[c];
        }
#pragma unroll
        for (int j = 0; j < kRawW; ++j) s_out[threadIdx.x * kRawW + j] = (float)acc[j];
    }
    __syncthreads();
    stage_rows<false>(s_out, grad_raw + p0 * kRawW, rows * kRawW);
}

void launch_appearance_fwd(const float* xyz, const float* raw, const GpuView* views, int n_views,
                           int64_t n_vp, float* opa_out, void* feat_out, bool bf16, hipStream_t s) {
    if (n_vp == 0) return;
    const dim3 grid((unsigned)((n_vp + kApBlock - 1) / kApBlock));
    if (bf16)
        hipLaunchKernelGGL(k_appearance_fwd<true>, grid, dim3(kApBlock), 0, s, xyz, raw, views, n_views, n_vp,
                           opa_out, feat_out);
    else
        hipLaunchKernelGGL(k_appearance_fwd<false>, grid, dim3(kApBlock), 0, s, xyz, raw, views, n_views, n_vp,
                           opa_out, feat_out);
}

void launch_appearance_bwd(const float* xyz, const float* raw, const GpuView* views, int n_views,
                           int64_t n_points, const float* g_opa, const float* g_feat, float* grad_raw,
                           hipStream_t s) {
    if (n_points == 0) return;
    hipLaunchKernelGGL(k_appearance_bwd, dim3((unsigned)((n_points + kApBlock - 1) / kApBlock)), dim3(kApBlock),
                       0, s, xyz, raw, views, n_views, n_points, g_opa, g_feat, grad_raw);
}

}  // namespace inpc
