// Tile-list blending (Eq. 1 with early termination, and its backward,
// Appendix A.6) for gfx950.
//
// Instead of one sorted list per pixel, the points are listed per square
// tile (16x16 or 8x8 pixels): one entry per (tile, point) pair for every tile
// the point's 2x2 footprint touches (about 1.13 or 1.27 entries per point),
// sorted stably by tile after the depth sort, so each tile's entries are in
// front-to-back order.  One block owns a tile, with L lanes per pixel.  The
// block walks its entries in chunks of one entry per thread: each thread
// reads one entry's point record and feature row (one payload row laid out
// by the projection; issued while the previous chunk is being blended),
// stores it into LDS and marks the pixels the entry covers in a per-pixel
// bit set.  With one lane per pixel, each thread then walks the set bits of
// its pixel in order; with L lanes, the lanes of a pixel first turn its bits
// into an ordered list of entry slots and then take L entries at a time,
// with the transmittance in front of each from a prefix product of
// 1 - alpha across the group (the grouped step of the per-pixel-list
// blend).  Restricted to one pixel, the entry order is the (depth, point)
// order of that pixel's splats, so the result is the per-pixel definition;
// with one lane per pixel the float32 operations are exactly those of the
// one-lane-per-pixel list blend.
#include "blend_common.h"

namespace inpc {

// TS x TS pixels per tile, L lanes per pixel, NT = TS * TS * L threads per
// block; one chunk = one entry per thread; NW words of entry bits per pixel.
template <int TS, int L>
struct TileDims {
    static constexpr int NPIX = TS * TS;
    static constexpr int NT = NPIX * L;
    static constexpr int NW = NT / 32;
};

struct TileCtx {
    const GpuView* V;
    uint32_t tile;     // global tile index
    int tx, ty;        // tile coordinates in its view
    int pix;           // pixel inside the tile (row-major)
    int lx, ly;
    int sub;           // lane within the pixel's group of L
    bool inside;
    int64_t q;         // packed pixel index
};

template <int TS, int L>
__device__ __forceinline__ TileCtx tile_ctx(const GpuView* __restrict__ views, int n_views,
                                            const uint32_t* __restrict__ perm) {
    TileCtx c;
    c.tile = perm[blockIdx.x];
    const int v = n_views == 1 ? 0
                               : find_view(views, n_views, (int64_t)c.tile,
                                           [](const GpuView& g) { return g.tile_offset; });
    c.V = views + v;
    const int64_t lt = (int64_t)c.tile - c.V->tile_offset;
    c.tx = (int)(lt % c.V->tiles_x);
    c.ty = (int)(lt / c.V->tiles_x);
    c.pix = (int)threadIdx.x / L;
    c.sub = (int)threadIdx.x % L;
    c.lx = c.pix % TS;
    c.ly = c.pix / TS;
    const int x = c.tx * TS + c.lx, y = c.ty * TS + c.ly;
    c.inside = x < c.V->W && y < c.V->H;
    c.q = c.V->pixel_offset + (int64_t)y * c.V->W + x;
    return c;
}

// LDS image of one chunk of entries: per entry a 16-byte geometry word
// (ax, ay, opacity, and the packed anchor word: tile-local x0+1, y0+1,
// corner mask; 0 = no entry), the view point, the feature row (rows of a
// multiple of 4 floats at a stride of FM + 4, read with 16-byte loads; other
// widths at an odd stride), the forward's T_k of the entry's four splats,
// for every pixel of the tile a bit per chunk entry that covers it, and
// (L > 1) every pixel's covering entry slots in order, at a row stride of
// NT + 4 bytes.
template <int TS, int L, int FM>
struct TileChunk {
    static constexpr int NT = TileDims<TS, L>::NT;
    static constexpr int NPIX = TileDims<TS, L>::NPIX;
    static constexpr bool VEC = FM % 4 == 0;
    static constexpr int FS = VEC ? FM + 4 : (FM | 1);   // feature row stride in floats
    static constexpr int BW = TileDims<TS, L>::NW + 1;   // words per pixel row of bits (odd stride)
    static constexpr int LS = L > 1 ? NT + 4 : 0;        // bytes per pixel row of entry slots
    float4 geo[NT];
    float4 tk[NT];
    float feat[NT * FS];
    uint32_t vp[NT];
    uint32_t bits[NPIX * BW];
    unsigned char lst[NPIX * LS + 4];
};

// Feature row of chunk entry j.
template <int TS, int L, int FM>
__device__ __forceinline__ void chunk_feat(const TileChunk<TS, L, FM>& S, int j, float (&v)[FM]) {
    constexpr int FS = TileChunk<TS, L, FM>::FS;
    if constexpr (TileChunk<TS, L, FM>::VEC) {
        const float4* r = reinterpret_cast<const float4*>(&S.feat[j * FS]);
#pragma unroll
        for (int i = 0; i < FM / 4; ++i) {
            const float4 q = r[i];
            v[4 * i] = q.x; v[4 * i + 1] = q.y; v[4 * i + 2] = q.z; v[4 * i + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int f = 0; f < FM; ++f) v[f] = S.feat[j * FS + f];
    }
}

__device__ __forceinline__ uint32_t geo_hit(const float4 g) { return __float_as_uint(g.w); }

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
                                            const float4* __restrict__ t_ent) {
    const uint32_t j = c0 + threadIdx.x;
    e.valid = c0 < end && j < end;
    if (e.valid) {
        e.vp = vals[j];
        const unsigned char* row = payload + (size_t)e.vp * ps;
        e.r = *reinterpret_cast<const PointRec*>(row);
        payload_feat<FT, FM, DYN>(reinterpret_cast<const FT*>(row + sizeof(PointRec)), Fd, e.cf);
        if constexpr (WANT_T) e.t4 = t_ent[j];
    }
}

// The two halves of fetch_entry for the software-pipelined chunk loops: a
// chunk's view points are loaded one chunk before its payload rows, so each
// chunk waits on one memory latency instead of two dependent ones.  Both
// loads are issued by every lane (indices past ``end`` are clamped to the
// tile's last entry, whose row is a real one): a load that some paths skip
// would make the compiler wait for every older memory operation instead of
// the ones it needs.  The tile must be non-empty (lo < end) in entry_vp_in.
__device__ __forceinline__ uint32_t entry_vp_in(uint32_t c0, uint32_t end, const uint32_t* __restrict__ vals) {
    const uint32_t j = c0 + threadIdx.x;
    return vals[j < end ? j : end - 1u];
}

template <typename FT, int FM, bool DYN, bool WANT_T>
__device__ __forceinline__ void fetch_entry_of(EntryRegs<FM>& e, uint32_t vp, uint32_t c0, uint32_t end,
                                               const unsigned char* __restrict__ payload, int ps, int Fd,
                                               const float4* __restrict__ t_ent) {
    const uint32_t j = c0 + threadIdx.x;
    e.valid = c0 < end && j < end;
    e.vp = vp;
    const unsigned char* row = payload + (size_t)vp * ps;
    e.r = *reinterpret_cast<const PointRec*>(row);
    payload_feat<FT, FM, DYN>(reinterpret_cast<const FT*>(row + sizeof(PointRec)), Fd, e.cf);
    if constexpr (WANT_T) e.t4 = t_ent[j < end ? j : end - 1u];
}

// Thread i stores its entry and marks the (at most four) pixels of the tile
// its splats cover; ``bits`` must be cleared before.  Every lane writes its
// slot (an invalid entry covers no pixel), without a branch around the use of
// the loaded values, so the compiler's wait for them holds on every path.
template <int TS, int L, int FM, bool WANT_T>
__device__ __forceinline__ void store_entry(TileChunk<TS, L, FM>& S, const TileCtx& c, const EntryRegs<FM>& e) {
    constexpr int FS = TileChunk<TS, L, FM>::FS, BW = TileChunk<TS, L, FM>::BW;
    const int i = threadIdx.x;
    if constexpr (TileChunk<TS, L, FM>::VEC) {
        float4* r = reinterpret_cast<float4*>(&S.feat[i * FS]);
#pragma unroll
        for (int q = 0; q < FM / 4; ++q)
            r[q] = make_float4(e.cf[4 * q], e.cf[4 * q + 1], e.cf[4 * q + 2], e.cf[4 * q + 3]);
    } else {
#pragma unroll
        for (int f = 0; f < FM; ++f) S.feat[i * FS + f] = e.cf[f];
    }
    if constexpr (WANT_T) S.tk[i] = e.t4;
    S.vp[i] = e.vp;
    const int lx0 = anc_x0(e.r.anc) - c.tx * TS, ly0 = anc_y0(e.r.anc) - c.ty * TS;
    const uint32_t mask = e.valid ? anc_mask(e.r.anc) : 0u;
    const uint32_t w = e.valid ? (uint32_t)(lx0 + 1) | ((uint32_t)(ly0 + 1) << 5) | (mask << 10) : 0u;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
        const int px = lx0 + (cc & 1), py = ly0 + (cc >> 1);
        if (((mask >> cc) & 1u) && (unsigned)px < (unsigned)TS && (unsigned)py < (unsigned)TS)
            atomicOr(&S.bits[(py * TS + px) * BW + (i >> 5)], 1u << (i & 31));
    }
    S.geo[i] = make_float4(e.valid ? e.r.ax : 0.0f, e.valid ? e.r.ay : 0.0f, e.valid ? e.r.opa : 0.0f,
                           __uint_as_float(w));
}

template <int TS, int L, int FM>
__device__ __forceinline__ void clear_bits(TileChunk<TS, L, FM>& S) {
    constexpr int NT = TileDims<TS, L>::NT, N = TileChunk<TS, L, FM>::NPIX * TileChunk<TS, L, FM>::BW;
#pragma unroll
    for (int k = 0; k < (N + NT - 1) / NT; ++k)
        if (k * NT + (int)threadIdx.x < N) S.bits[k * NT + threadIdx.x] = 0u;
}

// Corner of entry word w whose pixel is (lx, ly) (the entry covers it).
__device__ __forceinline__ int corner_of(uint32_t w, int lx, int ly) {
    const int dx = lx - ((int)(w & 31u) - 1), dy = ly - ((int)((w >> 5) & 31u) - 1);
    return (dy << 1) | dx;
}

// Keeps the bits of the entries j < lim of word wd.
__device__ __forceinline__ uint32_t below_lim(uint32_t m, int wd, int lim) {
    const int lo = wd * 32;
    if (lim <= lo) return 0u;
    if (lim < lo + 32) return m & ((1u << (lim - lo)) - 1u);
    return m;
}

// Bits of the entries j < lim of this chunk that cover the thread's pixel.
template <int TS, int L, int FM>
__device__ __forceinline__ uint32_t cover_word(const TileChunk<TS, L, FM>& S, const TileCtx& c, int wd, int lim) {
    return below_lim(S.bits[c.pix * TileChunk<TS, L, FM>::BW + wd], wd, lim);
}

// L > 1: the lanes of a pixel turn its cover bits of the entries j < lim
// into the ordered list of those entry slots (each lane takes NW / L words,
// placed by an exclusive prefix of their bit counts across the group) and
// clear every bit word of the pixel.  Returns the list length.
template <int TS, int L, int FM>
__device__ __forceinline__ int compact_cover(TileChunk<TS, L, FM>& S, const TileCtx& c, int lim) {
    constexpr int NW = TileDims<TS, L>::NW, WPL = NW / L, BW = TileChunk<TS, L, FM>::BW;
    static_assert(NW % L == 0 && TileDims<TS, L>::NT <= 256, "slot lists hold byte indices");
    uint32_t w[WPL];
    int cnt = 0;
#pragma unroll
    for (int t = 0; t < WPL; ++t) {
        const int wd = c.sub * WPL + t;
        uint32_t* b = &S.bits[c.pix * BW + wd];
        w[t] = below_lim(*b, wd, lim);
        *b = 0u;
        cnt += __popc(w[t]);
    }
    int inc = cnt;
#pragma unroll
    for (int d = 1; d < L; d <<= 1) {
        const int t = __shfl_up(inc, d, L);
        if (c.sub >= d) inc += t;
    }
    const int total = __shfl(inc, L - 1, L);
    unsigned char* out = S.lst + c.pix * TileChunk<TS, L, FM>::LS + (inc - cnt);
#pragma unroll
    for (int t = 0; t < WPL; ++t) {
        uint32_t m = w[t];
        while (m != 0u) {
            *out++ = (unsigned char)((c.sub * WPL + t) * 32 + (__ffs(m) - 1));
            m &= m - 1u;
        }
    }
    return total;
}

// Forward state of the thread's pixel across the chunks of its tile.
template <int FM>
struct FwdAcc {
    float C[FM];       // this lane's share of the colour
    float T;
    uint32_t nb;       // splats blended
    uint32_t last;     // one past the last blended entry of the tile range (0: none)
    bool done, started;
};

template <int FM>
__device__ __forceinline__ void fwd_init(FwdAcc<FM>& a, bool done) {
#pragma unroll
    for (int f = 0; f < FM; ++f) a.C[f] = 0.0f;
    a.T = 1.0f;
    a.nb = 0u;
    a.last = 0u;
    a.done = done;
    a.started = false;
}

// Blends the chunk's entries j < lim that cover the thread's pixel, in order.
// L == 1: walks the pixel's bits (the one-lane float32 recurrence, operation
// for operation); L > 1: takes the n slots listed by compact_cover L at a
// time with the grouped transmittance step.  COLOUR: accumulate the colour
// and write the per-splat weights T_k alpha_k.  s_tk (LDS, four floats per
// chunk entry, by corner) receives T_k if given.
template <int TS, int L, int FM, bool COLOUR>
__device__ __forceinline__ void blend_chunk(const TileChunk<TS, L, FM>& S, const TileCtx& c, uint32_t c0, int lim,
                                            int n, float tau, FwdAcc<FM>& a, float* s_tk,
                                            float* __restrict__ splat_weight) {
    constexpr int NW = TileDims<TS, L>::NW;
    if constexpr (L == 1) {
#pragma unroll
        for (int wd = 0; wd < NW; ++wd) {
            uint32_t m = cover_word<TS, L, FM>(S, c, wd, lim);
            while (m != 0u && !a.done) {
                const int j = wd * 32 + (__ffs(m) - 1);
                m &= m - 1u;
                const float4 ge = S.geo[j];
                const int corner = corner_of(geo_hit(ge), c.lx, c.ly);
                float wx, wy, alpha, om;
                corner_factors(ge.x, ge.y, corner, wx, wy);
                splat_alpha(ge.z, wx, wy, alpha, om);
                const uint32_t id = 4u * S.vp[j] + (uint32_t)corner;
                if constexpr (COLOUR) {
                    const float ta = a.T * alpha;
                    float cf[FM];
                    chunk_feat(S, j, cf);
#pragma unroll
                    for (int f = 0; f < FM; ++f) a.C[f] = __builtin_fmaf(ta, cf[f], a.C[f]);
                    if (splat_weight) splat_weight[id] = ta;
                }
                if (s_tk) s_tk[4 * j + corner] = a.T;
                a.T = a.T * om;
                ++a.nb;
                a.last = c0 + (uint32_t)j + 1u;
                if (a.T < tau) a.done = true;
            }
        }
    } else {
        const unsigned char* lst = S.lst + c.pix * TileChunk<TS, L, FM>::LS;
        for (int base = 0; base < n && !a.done; base += L) {
            const int k = base + c.sub;
            const bool valid = k < n;
            const int j = valid ? (int)lst[k] : 0;
            float alpha = 0.0f, om = 1.0f;
            int corner = 0;
            if (valid) {
                const float4 ge = S.geo[j];
                corner = corner_of(geo_hit(ge), c.lx, c.ly);
                float wx, wy;
                corner_factors(ge.x, ge.y, corner, wx, wy);
                splat_alpha(ge.z, wx, wy, alpha, om);
            }
            const GroupStep g = group_step<L>(a.T, om, valid, !a.started && c.sub == 0, tau, c.sub);
            a.started = true;
            if (g.blended) {
                const uint32_t id = 4u * S.vp[j] + (uint32_t)corner;
                if constexpr (COLOUR) {
                    const float ta = g.tb * alpha;
                    float cf[FM];
                    chunk_feat(S, j, cf);
#pragma unroll
                    for (int f = 0; f < FM; ++f) a.C[f] = __builtin_fmaf(ta, cf[f], a.C[f]);
                    if (splat_weight) splat_weight[id] = ta;
                }
                if (s_tk) s_tk[4 * j + corner] = g.tb;
            }
            // the blended lanes are a prefix of the group, in list order
            const int gbase = __lane_id() - c.sub;
            const uint32_t mine = (uint32_t)((__ballot(g.blended) >> gbase) & ((1ull << L) - 1ull));
            if (mine) {
                a.nb += (uint32_t)__popc(mine);
                a.last = c0 + (uint32_t)__shfl(j, 31 - __clz(mine), L) + 1u;
            }
            a.T = g.t_next;
            if (g.done) a.done = true;
        }
    }
}

template <typename FT, int FM, bool DYN, int TS, int L>
__global__ __launch_bounds__(TS * TS * L) void k_tile_fwd(
    const GpuView* __restrict__ views, int n_views, const uint32_t* __restrict__ perm, const uint2* __restrict__ range,
    const uint32_t* __restrict__ vals, const unsigned char* __restrict__ payload, int ps, int Fd,
    float tau, float* __restrict__ image, float* __restrict__ t_final, PixelState* __restrict__ state,
    float4* __restrict__ t_ent, float* __restrict__ splat_weight) {
    constexpr int NT = TileDims<TS, L>::NT;
    __shared__ TileChunk<TS, L, FM> S;
    float* s_tk = t_ent ? reinterpret_cast<float*>(S.tk) : nullptr;
    const TileCtx c = tile_ctx<TS, L>(views, n_views, perm);
    const uint2 r = range[c.tile];
    FwdAcc<FM> a;
    fwd_init(a, !c.inside);
    EntryRegs<FM> e{};   // invalid entries keep defined (zero) values
    fetch_entry<FT, FM, DYN, false>(e, r.x, r.y, vals, payload, ps, Fd, nullptr);
    if constexpr (L > 1) {
        // from here on compact_cover clears the bits it has read
        clear_bits<TS, L, FM>(S);
        __syncthreads();
    }
    // The T_k of a chunk's entries are stored (by entry, coalesced) at the
    // start of the next chunk, before its loads are issued, so that the loads
    // are always the youngest memory operations and waiting for them waits
    // for nothing else.  Only the last chunk can be partial; it is stored
    // after the loop.
    uint32_t c_last = r.x;
    // One chunk: vcur holds the view points of the next chunk; returns the
    // ones of the chunk after it, and sets ``stop`` once every pixel of the
    // tile has terminated.
    bool stop = false;
    auto chunk = [&](uint32_t c0, uint32_t vcur) -> uint32_t {
        if constexpr (L == 1) {
            clear_bits<TS, L, FM>(S);
            __syncthreads();
        }
        store_entry<TS, L, FM, false>(S, c, e);
        if (s_tk) {
            if (c0 > r.x) t_ent[c0 - NT + threadIdx.x] = S.tk[threadIdx.x];
            S.tk[threadIdx.x] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        __syncthreads();
        c_last = c0;
        const uint32_t vnext = entry_vp_in(c0 + 2 * NT, r.y, vals);
        fetch_entry_of<FT, FM, DYN, false>(e, vcur, c0 + NT, r.y, payload, ps, Fd, nullptr);
        const int lim = (int)(r.y - c0);
        int n = 0;
        if constexpr (L > 1) {
            n = compact_cover<TS, L, FM>(S, c, lim);
            __syncthreads();
        }
        if (!a.done) blend_chunk<TS, L, FM, true>(S, c, c0, lim, n, tau, a, s_tk, splat_weight);
        stop = __syncthreads_and(a.done ? 1 : 0);
        return vnext;
    };
    uint32_t vn = r.x < r.y ? entry_vp_in(r.x + NT, r.y, vals) : 0u;
    for (uint32_t c0 = r.x; c0 < r.y && !stop; c0 += NT) vn = chunk(c0, vn);
    if (s_tk && r.x < r.y && c_last + threadIdx.x < r.y) t_ent[c_last + threadIdx.x] = S.tk[threadIdx.x];
#pragma unroll
    for (int mm = L / 2; mm >= 1; mm >>= 1) {
#pragma unroll
        for (int f = 0; f < FM; ++f) a.C[f] += __shfl_xor(a.C[f], mm, L);
    }
    if (c.inside && c.sub == 0) {
        f32_store<FM, DYN>(image, c.q, Fd, a.C);
        t_final[c.q] = a.T;
        PixelState st;
        st.n_blended = a.nb;
        st.pad0 = a.last;
        st.pad1 = st.pad2 = 0;
        state[c.q] = st;
    }
}

template <typename FT, int FM, bool DYN, int TS, int L>
__global__ __launch_bounds__(TS * TS * L) void k_tile_bwd(
    const GpuView* __restrict__ views, int n_views, const uint32_t* __restrict__ perm, const uint2* __restrict__ range,
    const uint32_t* __restrict__ vals, const unsigned char* __restrict__ payload, int ps, int Fd,
    float tau, const PixelState* __restrict__ state, const float* __restrict__ g_img,
    const float* __restrict__ g_t, float4* __restrict__ t_ent, int rebuild_t, float2* __restrict__ frec) {
    constexpr int NT = TileDims<TS, L>::NT, NW = TileDims<TS, L>::NW;
    __shared__ TileChunk<TS, L, FM> S;
    __shared__ uint32_t s_last;
    const TileCtx c = tile_ctx<TS, L>(views, n_views, perm);
    const uint2 r = range[c.tile];
    const uint32_t last = c.inside ? state[c.q].pad0 : 0u;
    if (threadIdx.x == 0) s_last = 0u;
    if constexpr (L > 1) clear_bits<TS, L, FM>(S);   // then kept clear by compact_cover
    __syncthreads();
    if (last && c.sub == 0) atomicMax(&s_last, last);
    if (rebuild_t) {
        // T_k by the forward's own recurrence (same operations, same order).
        FwdAcc<FM> a;
        fwd_init(a, !c.inside);
        EntryRegs<FM> e{};   // invalid entries keep defined (zero) values
        fetch_entry<FT, FM, DYN, false>(e, r.x, r.y, vals, payload, ps, Fd, nullptr);
        for (uint32_t c0 = r.x; c0 < r.y; c0 += NT) {
            if constexpr (L == 1) {
                clear_bits<TS, L, FM>(S);
                __syncthreads();
            }
            store_entry<TS, L, FM, false>(S, c, e);
            S.tk[threadIdx.x] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            __syncthreads();
            fetch_entry<FT, FM, DYN, false>(e, c0 + NT, r.y, vals, payload, ps, Fd, nullptr);
            const int lim = (int)(r.y - c0);
            int n = 0;
            if constexpr (L > 1) {
                n = compact_cover<TS, L, FM>(S, c, lim);
                __syncthreads();
            }
            if (!a.done)
                blend_chunk<TS, L, FM, false>(S, c, c0, lim, n, tau, a, reinterpret_cast<float*>(S.tk), nullptr);
            const bool all_done = __syncthreads_and(a.done ? 1 : 0);
            if (c0 + threadIdx.x < r.y) t_ent[c0 + threadIdx.x] = S.tk[threadIdx.x];
            if (all_done) break;
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
    EntryRegs<FM> e{};   // invalid entries keep defined (zero) values
    fetch_entry<FT, FM, DYN, true>(e, r.x + (n_chunks - 1) * NT, r.y, vals, payload, ps, Fd, t_ent);
    for (int k = (int)n_chunks - 1; k >= 0; --k) {
        const uint32_t c0 = r.x + (uint32_t)k * NT;
        __syncthreads();   // the previous chunk's LDS reads are done
        if constexpr (L == 1) {
            clear_bits<TS, L, FM>(S);
            __syncthreads();
        }
        store_entry<TS, L, FM, true>(S, c, e);
        __syncthreads();
        if (k > 0)
            fetch_entry<FT, FM, DYN, true>(e, c0 - NT, r.y, vals, payload, ps, Fd, t_ent);
        const int lim = last > c0 ? (int)(last - c0) : 0;
        if constexpr (L == 1) {
            if (lim > 0) {
#pragma unroll
                for (int wd = NW - 1; wd >= 0; --wd) {
                    uint32_t m = cover_word<TS, L, FM>(S, c, wd, lim);
                    while (m != 0u) {
                        const int b = 31 - __clz(m);
                        m &= ~(1u << b);
                        const int j = wd * 32 + b;
                        const float4 ge = S.geo[j];
                        const int corner = corner_of(geo_hit(ge), c.lx, c.ly);
                        float wx, wy;
                        corner_factors(ge.x, ge.y, corner, wx, wy);
                        const uint32_t id = 4u * S.vp[j] + (uint32_t)corner;
                        const double alpha = (double)ge.z * ((double)wx * (double)wy);
                        float cf[FM];
                        chunk_feat(S, j, cf);
                        double gc = 0.0;
#pragma unroll
                        for (int f = 0; f < FM; ++f) gc = __builtin_fma((double)g[f], (double)cf[f], gc);
                        // T_k of this corner: one LDS word at a computed address
                        const double Tk = (double)reinterpret_cast<const float*>(S.tk)[4 * j + corner];
                        frec[id] = make_float2((float)(Tk * (gc - Y)), (float)(Tk * alpha));
                        Y = __builtin_fma(1.0 - alpha, Y, alpha * gc);
                    }
                }
            }
        } else {
            const int n = compact_cover<TS, L, FM>(S, c, lim);
            __syncthreads();
            const unsigned char* lst = S.lst + c.pix * TileChunk<TS, L, FM>::LS;
            // groups of L slots from the end of the pixel's list, lanes in list order
            for (int base = n > 0 ? ((n - 1) / L) * L : -1; base >= 0; base -= L) {
                const int kk = base + c.sub;
                const bool valid = kk < n;
                double A = 0.0, B = 1.0, alpha = 0.0, gc = 0.0, Tk = 0.0;
                uint32_t id = 0;
                if (valid) {
                    const int j = (int)lst[kk];
                    const float4 ge = S.geo[j];
                    const int corner = corner_of(geo_hit(ge), c.lx, c.ly);
                    float wx, wy;
                    corner_factors(ge.x, ge.y, corner, wx, wy);
                    id = 4u * S.vp[j] + (uint32_t)corner;
                    alpha = (double)ge.z * ((double)wx * (double)wy);
                    float cf[FM];
                    chunk_feat(S, j, cf);
#pragma unroll
                    for (int f = 0; f < FM; ++f) gc = __builtin_fma((double)g[f], (double)cf[f], gc);
                    Tk = (double)reinterpret_cast<const float*>(S.tk)[4 * j + corner];
                    A = alpha * gc;
                    B = 1.0 - alpha;
                }
                // inclusive suffix composition of the maps Y -> A + B Y of lanes sub .. L-1
#pragma unroll
                for (int d = 1; d < L; d <<= 1) {
                    const double A2 = __shfl_down(A, d, L);
                    const double B2 = __shfl_down(B, d, L);
                    if (c.sub + d < L) {
                        A = __builtin_fma(B, A2, A);
                        B = B * B2;
                    }
                }
                double Ae = __shfl_down(A, 1, L), Be = __shfl_down(B, 1, L);
                if (c.sub == L - 1) {
                    Ae = 0.0;
                    Be = 1.0;
                }
                const double y_next = __builtin_fma(Be, Y, Ae);
                if (valid) frec[id] = make_float2((float)(Tk * (gc - y_next)), (float)(Tk * alpha));
                Y = __builtin_fma(__shfl(B, 0, L), Y, __shfl(A, 0, L));
            }
        }
    }
}

template <typename FT, int FM, bool DYN, int TS, int L>
static void tile_fwd_t(const GpuView* views, int n_views, int64_t n_tiles, const uint32_t* perm, const uint2* range,
                       const uint32_t* vals,
                       const unsigned char* payload, int ps, int Fd, float tau, float* image, float* t_final,
                       PixelState* state, float4* t_ent, float* splat_weight, hipStream_t s) {
    hipLaunchKernelGGL((k_tile_fwd<FT, FM, DYN, TS, L>), dim3((unsigned)n_tiles), dim3(TS * TS * L), 0, s, views,
                       n_views, perm, range, vals, payload, ps, Fd, tau, image, t_final, state, t_ent, splat_weight);
}

template <typename FT, int FM, bool DYN, int TS, int L>
static void tile_bwd_t(const GpuView* views, int n_views, int64_t n_tiles, const uint32_t* perm, const uint2* range,
                       const uint32_t* vals,
                       const unsigned char* payload, int ps, int Fd, float tau, const PixelState* state,
                       const float* g_img, const float* g_t, float4* t_ent, int rebuild_t, float2* frec,
                       hipStream_t s) {
    hipLaunchKernelGGL((k_tile_bwd<FT, FM, DYN, TS, L>), dim3((unsigned)n_tiles), dim3(TS * TS * L), 0, s, views,
                       n_views, perm, range, vals, payload, ps, Fd, tau, state, g_img, g_t, t_ent, rebuild_t, frec);
}

// Calls body.template operator()<TS, L>() for the tile shape.
template <typename Body>
static void dispatch_tile(int shape, Body&& body) {
    switch (shape) {
        case kTileShape16: body.template operator()<16, 1>(); break;
        case kTileShape8x4: body.template operator()<8, 4>(); break;
        case kTileShape8x2: body.template operator()<8, 2>(); break;
        default: body.template operator()<8, 1>(); break;
    }
}

void launch_tile_fwd(int F, int feat_dtype, int shape, const GpuView* views, int n_views, int64_t n_tiles,
                     const uint32_t* perm, const uint2* range, const uint32_t* vals, const unsigned char* payload, int ps,
                     float tau, float* image, float* t_final, PixelState* state, float4* t_ent,
                     float* splat_weight, hipStream_t s) {
    if (n_tiles == 0) return;
    dispatch_tile(shape, [&]<int TS, int L>() {
        dispatch_f(F, [&]<int FM, bool DYN>() {
            if (feat_dtype == 1)
                tile_fwd_t<__hip_bfloat16, FM, DYN, TS, L>(views, n_views, n_tiles, perm, range, vals, payload, ps, F, tau,
                                                           image, t_final, state, t_ent, splat_weight, s);
            else
                tile_fwd_t<float, FM, DYN, TS, L>(views, n_views, n_tiles, perm, range, vals, payload, ps, F, tau, image,
                                                  t_final, state, t_ent, splat_weight, s);
        });
    });
}

void launch_tile_bwd(int F, int feat_dtype, int shape, const GpuView* views, int n_views, int64_t n_tiles,
                     const uint32_t* perm, const uint2* range, const uint32_t* vals, const unsigned char* payload, int ps,
                     float tau, const PixelState* state, const float* g_img, const float* g_t,
                     float4* t_ent, int rebuild_t, float2* frec, hipStream_t s) {
    if (n_tiles == 0) return;
    dispatch_tile(shape, [&]<int TS, int L>() {
        dispatch_f(F, [&]<int FM, bool DYN>() {
            if (feat_dtype == 1)
                tile_bwd_t<__hip_bfloat16, FM, DYN, TS, L>(views, n_views, n_tiles, perm, range, vals, payload, ps, F, tau,
                                                           state, g_img, g_t, t_ent, rebuild_t, frec, s);
            else
                tile_bwd_t<float, FM, DYN, TS, L>(views, n_views, n_tiles, perm, range, vals, payload, ps, F, tau, state,
                                                  g_img, g_t, t_ent, rebuild_t, frec, s);
        });
    });
}

}  // namespace inpc
