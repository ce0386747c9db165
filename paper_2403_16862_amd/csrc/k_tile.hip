// Tile-list blending (Eq. 1 with early termination, and its backward,
// Appendix A.6) for gfx950.
//
// Instead of one sorted list per pixel, the points are listed per square
// tile (16x16 or 8x8 pixels): one entry per (tile, point) pair for every tile
// the point's 2x2 footprint touches (about 1.13 or 1.27 entries per point),
// sorted stably by tile after the depth sort, so each tile's entries are in
// front-to-back order.  One block owns a tile, one thread per pixel.  The
// block walks its entries in chunks of one entry per thread: each thread
// gathers one entry's point record and feature row (independent gathers, issued while
// the previous chunk is being blended), stores it into LDS and marks the
// pixels the entry covers in a per-pixel bit set; every thread then blends
// the covering entries of its pixel in order, from LDS.  Restricted to one pixel, the entry order is the (depth,
// point) order of that pixel's splats, so the result is the per-pixel
// definition exactly; with one thread per pixel the float32 operations are
// those of the one-lane-per-pixel list blend.
#include "blend_common.h"

namespace inpc {

// TS x TS pixels per tile, TS * TS threads per block, one chunk = one entry
// per thread; NW words of entry bits per pixel.
template <int TS>
struct TileDims {
    static constexpr int NT = TS * TS;
    static constexpr int NW = NT / 32;
};

struct TileCtx {
    const GpuView* V;
    uint32_t tile;     // global tile index
    int tx, ty;        // tile coordinates in its view
    int lx, ly;        // pixel inside the tile
    bool inside;
    int64_t q;         // packed pixel index
};

template <int TS>
__device__ __forceinline__ TileCtx tile_ctx(const GpuView* __restrict__ views, int n_views) {
    TileCtx c;
    c.tile = xcd_remap(blockIdx.x, gridDim.x);
    const int v = n_views == 1 ? 0
                               : find_view(views, n_views, (int64_t)c.tile,
                                           [](const GpuView& g) { return g.tile_offset; });
    c.V = views + v;
    const int64_t lt = (int64_t)c.tile - c.V->tile_offset;
    c.tx = (int)(lt % c.V->tiles_x);
    c.ty = (int)(lt / c.V->tiles_x);
    c.lx = threadIdx.x % TS;
    c.ly = threadIdx.x / TS;
    const int x = c.tx * TS + c.lx, y = c.ty * TS + c.ly;
    c.inside = x < c.V->W && y < c.V->H;
    c.q = c.V->pixel_offset + (int64_t)y * c.V->W + x;
    return c;
}

// LDS image of one chunk of entries: packed anchor word (tile-local x0+1,
// y0+1, corner mask; 0 = no entry), record fields, feature rows at an odd
// stride (entries read by different lanes then fall in different banks),
// the forward's T_k of the entry's four splats (backward only), and for
// every pixel of the tile a bit per chunk entry that covers it.
template <int TS, int FM>
struct TileChunk {
    static constexpr int NT = TileDims<TS>::NT;
    static constexpr int FS = FM | 1;                   // odd row stride in floats
    static constexpr int BW = TileDims<TS>::NW + 1;     // words per pixel row of bits (odd stride)
    uint32_t hit[NT];
    float ax[NT], ay[NT], opa[NT];
    uint32_t vp[NT];
    float feat[NT * FS];
    float4 tk[NT];
    uint32_t bits[NT * BW];
};

// One entry held in registers between its gather and its store into LDS,
// so that the gathers of the next chunk overlap the blending of this one.
template <int FM>
struct EntryRegs {
    bool valid;
    uint32_t vp;
    PointRec r;
    float cf[FM];
    float4 t4;
};

// Feature row stored after the 16-byte record in a payload row (16-byte aligned).
template <typename FT, int FM, bool DYN>
__device__ __forceinline__ void payload_feat(const FT* __restrict__ row, int Fd, float (&c)[FM]) {
    if constexpr (!DYN) {
        load_row<FM>(row, c);
    } else {
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

// Gathers one entry: its view point, and the point's record and feature row
// from the co-located payload (one or two cache lines per point).
template <typename FT, int FM, bool DYN, bool WANT_T>
__device__ __forceinline__ void fetch_entry(EntryRegs<FM>& e, uint32_t c0, uint32_t end,
                                            const uint32_t* __restrict__ vals,
                                            const unsigned char* __restrict__ payload, int ps, int Fd,
                                            const float* __restrict__ t_id) {
    const uint32_t j = c0 + threadIdx.x;
    e.valid = c0 < end && j < end;
    if (e.valid) {
        e.vp = vals[j];
        const unsigned char* row = payload + (size_t)e.vp * ps;
        e.r = *reinterpret_cast<const PointRec*>(row);
        payload_feat<FT, FM, DYN>(reinterpret_cast<const FT*>(row + sizeof(PointRec)), Fd, e.cf);
        if constexpr (WANT_T) e.t4 = reinterpret_cast<const float4*>(t_id)[e.vp];
    }
}

// Thread i stores its entry and marks the (at most four) pixels of the tile
// its splats cover; ``bits`` must be cleared before.
template <int TS, int FM, bool WANT_T>
__device__ __forceinline__ void store_entry(TileChunk<TS, FM>& S, const TileCtx& c, const EntryRegs<FM>& e) {
    constexpr int FS = TileChunk<TS, FM>::FS, BW = TileChunk<TS, FM>::BW;
    const int i = threadIdx.x;
    uint32_t w = 0;
    if (e.valid) {
#pragma unroll
        for (int f = 0; f < FM; ++f) S.feat[i * FS + f] = e.cf[f];
        if constexpr (WANT_T) S.tk[i] = e.t4;
        S.ax[i] = e.r.ax;
        S.ay[i] = e.r.ay;
        S.opa[i] = e.r.opa;
        S.vp[i] = e.vp;
        const int lx0 = anc_x0(e.r.anc) - c.tx * TS, ly0 = anc_y0(e.r.anc) - c.ty * TS;
        const uint32_t mask = anc_mask(e.r.anc);
        w = (uint32_t)(lx0 + 1) | ((uint32_t)(ly0 + 1) << 5) | (mask << 10);
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const int px = lx0 + (cc & 1), py = ly0 + (cc >> 1);
            if (((mask >> cc) & 1u) && (unsigned)px < (unsigned)TS && (unsigned)py < (unsigned)TS)
                atomicOr(&S.bits[(py * TS + px) * BW + (i >> 5)], 1u << (i & 31));
        }
    }
    S.hit[i] = w;
}

template <int TS, int FM>
__device__ __forceinline__ void clear_bits(TileChunk<TS, FM>& S) {
    constexpr int BW = TileChunk<TS, FM>::BW;
#pragma unroll
    for (int k = 0; k < BW; ++k) S.bits[threadIdx.x * BW + k] = 0u;
}

// Corner of entry word w whose pixel is (lx, ly) (the entry covers it).
__device__ __forceinline__ int corner_of(uint32_t w, int lx, int ly) {
    const int dx = lx - ((int)(w & 31u) - 1), dy = ly - ((int)((w >> 5) & 31u) - 1);
    return (dy << 1) | dx;
}

// Bits of the entries j < lim of this chunk that cover the thread's pixel.
template <int TS, int FM>
__device__ __forceinline__ uint32_t cover_word(const TileChunk<TS, FM>& S, int wd, int lim) {
    uint32_t m = S.bits[threadIdx.x * TileChunk<TS, FM>::BW + wd];
    const int lo = wd * 32;
    if (lim <= lo) m = 0u;
    else if (lim < lo + 32) m &= (1u << (lim - lo)) - 1u;
    return m;
}

template <typename FT, int FM, bool DYN, int TS>
__global__ __launch_bounds__(TS * TS) void k_tile_fwd(
    const GpuView* __restrict__ views, int n_views, const uint2* __restrict__ range,
    const uint32_t* __restrict__ vals, const unsigned char* __restrict__ payload, int ps, int Fd,
    float tau, float* __restrict__ image, float* __restrict__ t_final, PixelState* __restrict__ state,
    float* __restrict__ t_id, float* __restrict__ splat_weight) {
    constexpr int FS = TileChunk<TS, FM>::FS, NT = TileDims<TS>::NT, NW = TileDims<TS>::NW;
    __shared__ TileChunk<TS, FM> S;
    const TileCtx c = tile_ctx<TS>(views, n_views);
    const uint2 r = range[c.tile];
    float C[FM];
#pragma unroll
    for (int f = 0; f < FM; ++f) C[f] = 0.0f;
    float T = 1.0f;
    uint32_t nb = 0, last = 0;
    bool done = !c.inside;
    EntryRegs<FM> e;
    fetch_entry<FT, FM, DYN, false>(e, r.x, r.y, vals, payload, ps, Fd, nullptr);
    for (uint32_t c0 = r.x; c0 < r.y; c0 += NT) {
        clear_bits<TS, FM>(S);
        __syncthreads();
        store_entry<TS, FM, false>(S, c, e);
        __syncthreads();
        fetch_entry<FT, FM, DYN, false>(e, c0 + NT, r.y, vals, payload, ps, Fd, nullptr);
        if (!done) {
            const int lim = (int)(r.y - c0);
#pragma unroll
            for (int wd = 0; wd < NW; ++wd) {
                uint32_t m = cover_word<TS, FM>(S, wd, lim);
                while (m != 0u && !done) {
                    const int j = wd * 32 + (__ffs(m) - 1);
                    m &= m - 1u;
                    const int corner = corner_of(S.hit[j], c.lx, c.ly);
                    float wx, wy, alpha, om;
                    corner_factors(S.ax[j], S.ay[j], corner, wx, wy);
                    splat_alpha(S.opa[j], wx, wy, alpha, om);
                    const uint32_t id = 4u * S.vp[j] + (uint32_t)corner;
                    const float ta = T * alpha;
#pragma unroll
                    for (int f = 0; f < FM; ++f) C[f] = __builtin_fmaf(ta, S.feat[j * FS + f], C[f]);
                    if (t_id) t_id[id] = T;
                    if (splat_weight) splat_weight[id] = ta;
                    T = T * om;
                    ++nb;
                    last = c0 + (uint32_t)j + 1u;
                    if (T < tau) done = true;
                }
            }
        }
        if (__syncthreads_and(done ? 1 : 0)) break;
    }
    if (c.inside) {
        f32_store<FM, DYN>(image, c.q, Fd, C);
        t_final[c.q] = T;
        PixelState st;
        st.n_blended = nb;
        st.pad0 = last;   // one past the last blended entry (0: none)
        st.pad1 = st.pad2 = 0;
        state[c.q] = st;
    }
}

template <typename FT, int FM, bool DYN, int TS>
__global__ __launch_bounds__(TS * TS) void k_tile_bwd(
    const GpuView* __restrict__ views, int n_views, const uint2* __restrict__ range,
    const uint32_t* __restrict__ vals, const unsigned char* __restrict__ payload, int ps, int Fd,
    float tau, const PixelState* __restrict__ state, const float* __restrict__ g_img,
    const float* __restrict__ g_t, float* __restrict__ t_id, int rebuild_t, float2* __restrict__ frec) {
    constexpr int FS = TileChunk<TS, FM>::FS, NT = TileDims<TS>::NT, NW = TileDims<TS>::NW;
    __shared__ TileChunk<TS, FM> S;
    __shared__ uint32_t s_last;
    const TileCtx c = tile_ctx<TS>(views, n_views);
    const uint2 r = range[c.tile];
    const uint32_t last = c.inside ? state[c.q].pad0 : 0u;
    if (threadIdx.x == 0) s_last = 0u;
    __syncthreads();
    if (last) atomicMax(&s_last, last);
    if (rebuild_t) {
        // T_k by the forward's own recurrence (same operations, same order).
        float T = 1.0f;
        bool done = !c.inside;
        EntryRegs<FM> e;
        fetch_entry<FT, FM, DYN, false>(e, r.x, r.y, vals, payload, ps, Fd, nullptr);
        for (uint32_t c0 = r.x; c0 < r.y; c0 += NT) {
            clear_bits<TS, FM>(S);
            __syncthreads();
            store_entry<TS, FM, false>(S, c, e);
            __syncthreads();
            fetch_entry<FT, FM, DYN, false>(e, c0 + NT, r.y, vals, payload, ps, Fd, nullptr);
            if (!done) {
                const int lim = (int)(r.y - c0);
#pragma unroll
                for (int wd = 0; wd < NW; ++wd) {
                    uint32_t m = cover_word<TS, FM>(S, wd, lim);
                    while (m != 0u && !done) {
                        const int j = wd * 32 + (__ffs(m) - 1);
                        m &= m - 1u;
                        const int corner = corner_of(S.hit[j], c.lx, c.ly);
                        float wx, wy, alpha, om;
                        corner_factors(S.ax[j], S.ay[j], corner, wx, wy);
                        splat_alpha(S.opa[j], wx, wy, alpha, om);
                        t_id[4u * S.vp[j] + (uint32_t)corner] = T;
                        T = T * om;
                        if (T < tau) done = true;
                    }
                }
            }
            if (__syncthreads_and(done ? 1 : 0)) break;
        }
        // the T_k written above are read back through the chunk loads below
        __threadfence_block();
    }
    __syncthreads();
    const uint32_t lmax = s_last;
    if (lmax == 0u) return;   // nothing blended in this tile (uniform across the block)
    float g[FM];
    double Y = 0.0;
    if (c.inside) {
        f32_row<FM, DYN>(g_img, c.q, Fd, g);
        Y = g_t ? (double)g_t[c.q] : 0.0;
    } else {
#pragma unroll
        for (int f = 0; f < FM; ++f) g[f] = 0.0f;
    }
    const uint32_t n_chunks = (lmax - r.x + NT - 1) / NT;
    EntryRegs<FM> e;
    fetch_entry<FT, FM, DYN, true>(e, r.x + (n_chunks - 1) * NT, r.y, vals, payload, ps, Fd, t_id);
    for (int k = (int)n_chunks - 1; k >= 0; --k) {
        const uint32_t c0 = r.x + (uint32_t)k * NT;
        __syncthreads();   // the previous chunk's LDS reads are done
        clear_bits<TS, FM>(S);
        __syncthreads();
        store_entry<TS, FM, true>(S, c, e);
        __syncthreads();
        if (k > 0)
            fetch_entry<FT, FM, DYN, true>(e, c0 - NT, r.y, vals, payload, ps, Fd, t_id);
        if (last > c0) {
            const int lim = (int)(last - c0);
#pragma unroll
            for (int wd = NW - 1; wd >= 0; --wd) {
                uint32_t m = cover_word<TS, FM>(S, wd, lim);
                while (m != 0u) {
                    const int b = 31 - __clz(m);
                    m &= ~(1u << b);
                    const int j = wd * 32 + b;
                    const int corner = corner_of(S.hit[j], c.lx, c.ly);
                    float wx, wy;
                    corner_factors(S.ax[j], S.ay[j], corner, wx, wy);
                    const uint32_t id = 4u * S.vp[j] + (uint32_t)corner;
                    const double alpha = (double)S.opa[j] * ((double)wx * (double)wy);
                    double gc = 0.0;
#pragma unroll
                    for (int f = 0; f < FM; ++f) gc = __builtin_fma((double)g[f], (double)S.feat[j * FS + f], gc);
                    const float4 t4 = S.tk[j];
                    const double Tk = (double)(corner == 0 ? t4.x : corner == 1 ? t4.y : corner == 2 ? t4.z : t4.w);
                    frec[id] = make_float2((float)(Tk * (gc - Y)), (float)(Tk * alpha));
                    Y = __builtin_fma(1.0 - alpha, Y, alpha * gc);
                }
            }
        }
    }
}

template <typename FT, int FM, bool DYN, int TS>
static void tile_fwd_t(const GpuView* views, int n_views, int64_t n_tiles, const uint2* range, const uint32_t* vals,
                       const unsigned char* payload, int ps, int Fd, float tau, float* image, float* t_final,
                       PixelState* state, float* t_id, float* splat_weight, hipStream_t s) {
    hipLaunchKernelGGL((k_tile_fwd<FT, FM, DYN, TS>), dim3((unsigned)n_tiles), dim3(TS * TS), 0, s, views, n_views,
                       range, vals, payload, ps, Fd, tau, image, t_final, state, t_id,
                       splat_weight);
}

template <typename FT, int FM, bool DYN, int TS>
static void tile_bwd_t(const GpuView* views, int n_views, int64_t n_tiles, const uint2* range, const uint32_t* vals,
                       const unsigned char* payload, int ps, int Fd, float tau, const PixelState* state,
                       const float* g_img, const float* g_t, float* t_id, int rebuild_t, float2* frec,
                       hipStream_t s) {
    hipLaunchKernelGGL((k_tile_bwd<FT, FM, DYN, TS>), dim3((unsigned)n_tiles), dim3(TS * TS), 0, s, views, n_views,
                       range, vals, payload, ps, Fd, tau, state, g_img, g_t, t_id,
                       rebuild_t, frec);
}

void launch_tile_fwd(int F, int feat_dtype, int shape, const GpuView* views, int n_views, int64_t n_tiles,
                     const uint2* range, const uint32_t* vals, const unsigned char* payload, int ps,
                     float tau, float* image, float* t_final, PixelState* state, float* t_id,
                     float* splat_weight, hipStream_t s) {
    if (n_tiles == 0) return;
    auto go = [&]<int TS>() {
        dispatch_f(F, [&]<int FM, bool DYN>() {
            if (feat_dtype == 1)
                tile_fwd_t<__hip_bfloat16, FM, DYN, TS>(views, n_views, n_tiles, range, vals, payload, ps, F, tau,
                                                        image, t_final, state, t_id, splat_weight, s);
            else
                tile_fwd_t<float, FM, DYN, TS>(views, n_views, n_tiles, range, vals, payload, ps, F, tau, image,
                                               t_final, state, t_id, splat_weight, s);
        });
    };
    if (tile_size_of(shape) == 16) go.template operator()<16>();
    else go.template operator()<8>();
}

void launch_tile_bwd(int F, int feat_dtype, int shape, const GpuView* views, int n_views, int64_t n_tiles,
                     const uint2* range, const uint32_t* vals, const unsigned char* payload, int ps,
                     float tau, const PixelState* state, const float* g_img, const float* g_t,
                     float* t_id, int rebuild_t, float2* frec, hipStream_t s) {
    if (n_tiles == 0) return;
    auto go = [&]<int TS>() {
        dispatch_f(F, [&]<int FM, bool DYN>() {
            if (feat_dtype == 1)
                tile_bwd_t<__hip_bfloat16, FM, DYN, TS>(views, n_views, n_tiles, range, vals, payload, ps, F, tau,
                                                        state, g_img, g_t, t_id, rebuild_t, frec, s);
            else
                tile_bwd_t<float, FM, DYN, TS>(views, n_views, n_tiles, range, vals, payload, ps, F, tau, state,
                                               g_img, g_t, t_id, rebuild_t, frec, s);
        });
    };
    if (tile_size_of(shape) == 16) go.template operator()<16>();
    else go.template operator()<8>();
}

}  // namespace inpc
