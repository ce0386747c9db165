// Projection / culling (Section 3.4, Eq. 5) and bilinear splat emission
// (Section 3.4, Eq. 6; the BilinearSplatting and ExclusiveSum steps of
// Algorithm 1) for gfx950.
#include "internal.h"

namespace inpc {

// ------------------------------------------------------------- view upload
constexpr int kUploadChunk = 16;
struct ViewChunk {
    GpuView v[kUploadChunk];
};

__global__ void k_upload_views(ViewChunk chunk, int n, GpuView* __restrict__ dst) {
    // One thread per 16-byte word of the chunk.
    const int words = n * (int)(sizeof(GpuView) / 16);
    const int i = threadIdx.x;
    if (i < words) reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(chunk.v)[i];
}

void launch_upload_views(const GpuView* host_views, int n, GpuView* dev, hipStream_t s) {
    for (int base = 0; base < n; base += kUploadChunk) {
        ViewChunk c{};
        const int k = (n - base) < kUploadChunk ? (n - base) : kUploadChunk;
        for (int i = 0; i < k; ++i) c.v[i] = host_views[base + i];
        hipLaunchKernelGGL(k_upload_views, dim3(1), dim3(kUploadChunk * sizeof(GpuView) / 16), 0, s,
                           c, k, dev + base);
    }
}

// --------------------------------------------------------------------- fill
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x * 4;
    for (size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n; i += stride) {
        if (i + 4 <= n) {
            reinterpret_cast<uint4*>(p + i)[0] = make_uint4(value, value, value, value);
        } else {
            for (size_t j = i; j < n; ++j) p[j] = value;
        }
    }
}

void launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t s) {
    if (n == 0) return;
    size_t blocks = (n / 4 + 255) / 256 + 1;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, value, n);
}

// --------------------------------------------------------------- projection
// The float32 operations below decide which splats exist and where, so they
// are evaluated exactly as written: no contraction into fused multiply-adds,
// correctly rounded division, and this association order.
// Number of distinct 2^lg x 2^lg tiles among the pixels of the corners in mask.
__device__ __forceinline__ uint32_t tile_entries(int x0, int y0, uint32_t mask, int lg) {
    uint32_t t[4];
    uint32_t n = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        if (!((mask >> c) & 1u)) continue;
        const uint32_t k = ((uint32_t)((y0 + (c >> 1)) >> lg) << 16) | (uint32_t)((x0 + (c & 1)) >> lg);
        bool dup = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) dup |= (j < (int)n) && t[j] == k;
        if (!dup) t[n++] = k;
    }
    return n;
}

__device__ __forceinline__ void project_point(const GpuView& V, float x, float y, float z,
                                              PointRec& r, uint32_t& zbits) {
#pragma clang fp contract(off)
    const float xc = ((V.R[0] * x + V.R[1] * y) + V.R[2] * z) + V.t[0];
    const float yc = ((V.R[3] * x + V.R[4] * y) + V.R[5] * z) + V.t[1];
    const float zc = ((V.R[6] * x + V.R[7] * y) + V.R[8] * z) + V.t[2];
    r.ax = 0.0f;
    r.ay = 0.0f;
    r.anc = 0u;
    zbits = kCulledKey;
    if (!(zc > V.near_p && zc < V.far_p)) return;
    const float u = V.fx * (xc / zc) + V.cx;
    const float v = V.fy * (yc / zc) + V.cy;
    if (!(u > -1.0f && u < (float)(V.W + 1))) return;
    if (!(v > -1.0f && v < (float)(V.H + 1))) return;
    const float su = u - 0.5f, sv = v - 0.5f;
    const float fx0 = floorf(su), fy0 = floorf(sv);
    const int x0 = (int)fx0, y0 = (int)fy0;
    const float ax = su - (float)x0, ay = sv - (float)y0;
    const float wx0 = 1.0f - ax, wy0 = 1.0f - ay;
    uint32_t mask = 0;
    const bool col0 = x0 >= 0 && x0 < V.W && wx0 > 0.0f;
    const bool col1 = x0 + 1 >= 0 && x0 + 1 < V.W && ax > 0.0f;
    const bool row0 = y0 >= 0 && y0 < V.H && wy0 > 0.0f;
    const bool row1 = y0 + 1 >= 0 && y0 + 1 < V.H && ay > 0.0f;
    mask |= (col0 && row0) ? 1u : 0u;
    mask |= (col1 && row0) ? 2u : 0u;
    mask |= (col0 && row1) ? 4u : 0u;
    mask |= (col1 && row1) ? 8u : 0u;
    if (mask == 0u) return;
    r.ax = ax;
    r.ay = ay;
    r.anc = (uint32_t)(x0 + 1) | ((uint32_t)(y0 + 1) << 14) | (mask << 28);
    zbits = __float_as_uint(zc);
}

// One block's run of payload rows (CPR 16-byte pieces per row, 256 rows):
// thread t writes piece t % CPR of rows t / CPR, t / CPR + 256 / CPR, ...
// All of the thread's feature pieces are requested before the first store,
// and unconditionally (a padding piece, or a row without splats, reads a
// real piece of its row, or of feature row 0, and drops it), so that the
// thread waits on one memory latency instead of one per row.
template <int CPR>
__device__ __forceinline__ void payload_run(uint4* __restrict__ dst, const PointRec* s_rec, const int64_t* s_row,
                                            int rows, const unsigned char* __restrict__ feat, int frow) {
    static_assert(CPR == 4 || CPR == 8, "pieces per payload row");
    constexpr int RSTEP = 256 / CPR;
    const int fcs = frow / 16;   // feature pieces per row (>= 1)
    const int col = (int)threadIdx.x % CPR, row0 = (int)threadIdx.x / CPR;
    const int fc = col < 1 ? 1 : (col > fcs ? fcs : col);
    auto ld = [&](int k) -> uint4 {
        const int row = row0 + k * RSTEP;
        const int64_t ar = row < rows ? s_row[row] : -1;
        return reinterpret_cast<const uint4*>(feat + (size_t)(ar >= 0 ? ar : 0) * frow)[fc - 1];
    };
    auto st = [&](int k, uint4 g) {
        const int row = row0 + k * RSTEP;
        if (row < rows && s_row[row] >= 0) {
            // selects on values (a select of addresses would put g in private memory)
            const PointRec rr = s_rec[row];
            const bool pad = col > fcs, rec = col == 0;
            uint4 v;
            v.x = rec ? __float_as_uint(rr.ax) : (pad ? 0u : g.x);
            v.y = rec ? __float_as_uint(rr.ay) : (pad ? 0u : g.y);
            v.z = rec ? __float_as_uint(rr.opa) : (pad ? 0u : g.z);
            v.w = rec ? rr.anc : (pad ? 0u : g.w);
            dst[row * CPR + col] = v;
        }
    };
    // named values rather than an array, which the compiler would keep in scratch
    const uint4 g0 = ld(0), g1 = ld(1), g2 = ld(2), g3 = ld(3);
    if constexpr (CPR == 8) {
        const uint4 g4 = ld(4), g5 = ld(5), g6 = ld(6), g7 = ld(7);
        st(0, g0); st(1, g1); st(2, g2); st(3, g3); st(4, g4); st(5, g5); st(6, g6); st(7, g7);
    } else {
        st(0, g0); st(1, g1); st(2, g2); st(3, g3);
    }
}

// Depth keys are float32 bits of z minus the bits of the smallest near
// plane (z > near >= 0 and bits are monotone there), so they need only as
// many bits as the (near, far) range spans; points without splats get
// zkey_none, which is larger than every real key.
__global__ __launch_bounds__(256) void k_project(const float* __restrict__ xyz,
                                                 const float* __restrict__ opacity,
                                                 const GpuView* __restrict__ views, int n_views,
                                                 int64_t n_vp, uint32_t zbase, uint32_t zkey_none,
                                                 PointRec* __restrict__ rec,
                                                 uint32_t* __restrict__ zkey,
                                                 uint32_t* __restrict__ zval,
                                                 uint32_t* __restrict__ zanc, int tile_log2,
                                                 const unsigned char* __restrict__ feat, int frow,
                                                 unsigned char* __restrict__ payload, int ps) {
    __shared__ PointRec s_rec[256];
    __shared__ int64_t s_row[256];   // feature row of the view point, -1 when no payload is due
    const int64_t vp0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t vp = vp0 + threadIdx.x;
    int64_t arow = -1;
    PointRec r{};
    // In a batch, the block's view is looked up once (uniform, scalar
    // loads); a block that straddles two views searches per thread.  (With
    // one view the per-thread form measures a little faster.)
    auto vstart = [](const GpuView& g) { return g.vpoint_offset; };
    const int v0 = n_views == 1 ? 0 : find_view(views, n_views, vp0, vstart);
    const bool one_view = n_views > 1 && vp0 + 256 <= views[v0].vpoint_offset + views[v0].point_count;
    auto point = [&](const GpuView& V) {
        const int64_t p = V.point_offset + (vp - V.vpoint_offset);
        arow = V.attr_offset + (vp - V.vpoint_offset);
        const float x = xyz[3 * p], y = xyz[3 * p + 1], z = xyz[3 * p + 2];
        const float o = opacity[arow];
        uint32_t zb;
        project_point(V, x, y, z, r, zb);
        r.opa = o;
        return zb;
    };
    if (vp < n_vp) {
        uint32_t zb;
        if (one_view) zb = point(views[v0]);
        else zb = point(views[n_views == 1 ? 0 : find_view(views, n_views, vp, vstart)]);
        rec[vp] = r;
        zkey[vp] = r.anc != 0u ? zb - zbase : zkey_none;
        const uint32_t m = anc_mask(r.anc);
        const uint32_t hb = tile_log2 ? (m ? tile_entries(anc_x0(r.anc), anc_y0(r.anc), m, tile_log2) : 0u) : m;
        zval[vp] = (uint32_t)vp | (hb << 28);
        zanc[vp] = r.anc;
        if (!m) arow = -1;
    }
    if (!payload) return;
    if ((frow & 15) == 0) {
        // The block's payload rows are one contiguous run: write it with
        // consecutive threads on consecutive 16-byte pieces (record from LDS,
        // feature pieces straight from the feature rows).
        s_rec[threadIdx.x] = r;
        s_row[threadIdx.x] = arow;
        __syncthreads();
        const int64_t rows64 = n_vp - vp0;
        const int rows = rows64 < 256 ? (int)rows64 : 256;
        // Whole 16-byte pieces of every due row are written, padding included
        // (zeros), so no cache line of the payload is left partly written.
        const int cpr = ps / 16, fcs = frow / 16;
        uint4* dst = reinterpret_cast<uint4*>(payload + (size_t)vp0 * ps);
        auto piece = [&](int row, int col) -> uint4 {
            if (col == 0) return *reinterpret_cast<const uint4*>(&s_rec[row]);
            if (col <= fcs) return reinterpret_cast<const uint4*>(feat + (size_t)s_row[row] * frow)[col - 1];
            return make_uint4(0u, 0u, 0u, 0u);
        };
        if (cpr == 4) {
            payload_run<4>(dst, s_rec, s_row, rows, feat, frow);
        } else if (cpr == 8) {
            payload_run<8>(dst, s_rec, s_row, rows, feat, frow);
        } else if ((256 % cpr) == 0) {
            const int col = threadIdx.x % cpr, rstep = 256 / cpr;
            for (int row = threadIdx.x / cpr; row < rows; row += rstep)
                if (s_row[row] >= 0) dst[row * cpr + col] = piece(row, col);
        } else {
            for (int k = threadIdx.x; k < rows * cpr; k += 256) {
                const int row = k / cpr, col = k - row * cpr;
                if (s_row[row] >= 0) dst[k] = piece(row, col);
            }
        }
    } else if (arow >= 0) {
        unsigned char* d = payload + (size_t)vp * ps;
        reinterpret_cast<PointRec*>(d)[0] = r;
        const unsigned char* src = feat + (size_t)arow * frow;
        d += sizeof(PointRec);
        if ((frow & 3) == 0) {
            for (int b = 0; b < frow; b += 4)
                *reinterpret_cast<uint32_t*>(d + b) = *reinterpret_cast<const uint32_t*>(src + b);
        } else {
            for (int b = 0; b < frow; b += 2)
                *reinterpret_cast<uint16_t*>(d + b) = *reinterpret_cast<const uint16_t*>(src + b);
        }
    }
}

void launch_project(const float* xyz, const float* opa, const GpuView* views, int n_views,
                    int64_t n_vp, uint32_t zbase, uint32_t zkey_none, PointRec* rec, uint32_t* zkey,
                    uint32_t* zval, uint32_t* zanc, int tile_log2, const void* feat, int feat_row_bytes,
                    unsigned char* payload, int ps, hipStream_t s) {
    if (n_vp == 0) return;
    const int64_t blocks = (n_vp + 255) / 256;
    hipLaunchKernelGGL(k_project, dim3((unsigned)blocks), dim3(256), 0, s, xyz, opa, views, n_views,
                       n_vp, zbase, zkey_none, rec, zkey, zval, zanc, tile_log2,
                       reinterpret_cast<const unsigned char*>(feat), feat_row_bytes, payload, ps);
}

// ----------------------------------------------------------------- emission
constexpr int kLdsViews = 64;   // views whose tile placement the tile emission keeps in LDS

// Fragments are emitted in the order of the depth-sorted points, corners in
// ascending order, so the emitted sequence is ordered by (depth, splat id).
// Count -> exclusive scan of chunk counts -> order-preserving write.  Each
// point's anchor word travels with it through the depth sort, so the write
// reads it in sorted order instead of gathering it by view point (one
// 128-byte line per point).
constexpr int kChunk = kEmitBlock * kEmitItems;

size_t emit_chunks(int64_t n_vp) { return (size_t)((n_vp + kChunk - 1) / kChunk); }

// Sorted view points that take part: the depth sort leaves out the points
// without splats and writes how many it kept to *n_live (at most n_vp).
__device__ __forceinline__ int64_t live_points(const uint32_t* n_live, int64_t n_vp) {
    if (!n_live) return n_vp;
    const int64_t n = (int64_t)*n_live;
    return n < n_vp ? n : n_vp;
}

// Items per view point: the corner count (popcount of the mask) or, for tile
// entries, the count itself.
template <bool TILE>
__device__ __forceinline__ uint32_t items_of(uint32_t zval) {
    return TILE ? (zval >> 28) : (uint32_t)__popc(zval >> 28);
}

// Besides counting, the blocks clear ``clear_words`` words at ``clear`` (the
// range array the ranges kernel fills after the sort), so no separate fill
// launch is needed.
template <bool TILE>
__global__ __launch_bounds__(kEmitBlock) void k_emit_count(const uint32_t* __restrict__ zval,
                                                           int64_t n_vp,
                                                           const uint32_t* __restrict__ n_live,
                                                           uint32_t* __restrict__ chunk_cnt,
                                                           uint32_t* __restrict__ clear, size_t clear_words) {
    __shared__ uint32_t s_tmp[kEmitBlock / kWave];
    {
        const size_t stride = (size_t)gridDim.x * kEmitBlock * 4;
        for (size_t i = ((size_t)blockIdx.x * kEmitBlock + threadIdx.x) * 4; i < clear_words; i += stride) {
            if (i + 4 <= clear_words) {
                reinterpret_cast<uint4*>(clear + i)[0] = make_uint4(0u, 0u, 0u, 0u);
            } else {
                for (size_t j = i; j < clear_words; ++j) clear[j] = 0u;
            }
        }
    }
    const int64_t live = live_points(n_live, n_vp);
    const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kEmitItems;
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < kEmitItems; ++i)
        if (base + i < live) cnt += items_of<TILE>(zval[base + i]);
    uint32_t total;
    block_excl_sum<kEmitBlock>(cnt, total, s_tmp);
    if (threadIdx.x == 0) chunk_cnt[blockIdx.x] = total;
}

// Exclusive scan of the chunk counts in one block; writes the total (the
// fragment count M) to m_dev[0] and the layout code of the lists to m_dev[1].
__global__ __launch_bounds__(1024) void k_scan_chunks(uint32_t* __restrict__ cnt, size_t n,
                                                      uint32_t* __restrict__ m_dev, uint32_t layout) {
    // 8 consecutive counts per thread, so that one round (two barriers)
    // covers 8192 chunks (8M view points) instead of 1024
    constexpr int K = 8;
    __shared__ uint32_t s_tmp[1024 / kWave];
    uint32_t running = 0;
    for (size_t base = 0; base < n; base += 1024 * K) {
        const size_t i0 = base + (size_t)threadIdx.x * K;
        uint32_t x[K], sum = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            x[k] = i0 + k < n ? cnt[i0 + k] : 0u;
            sum += x[k];
        }
        uint32_t total;
        uint32_t ex = running + block_excl_sum<1024>(sum, total, s_tmp);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (i0 + k < n) cnt[i0 + k] = ex;
            ex += x[k];
        }
        running += total;
    }
    if (threadIdx.x == 0) {
        m_dev[0] = running;
        m_dev[1] = layout;
    }
}

__global__ __launch_bounds__(kEmitBlock) void k_emit_write(
    const uint32_t* __restrict__ zval, const uint32_t* __restrict__ zanc,
    const GpuView* __restrict__ views, int n_views, int64_t n_vp, const uint32_t* __restrict__ n_live,
    const uint32_t* __restrict__ chunk_off, uint32_t* __restrict__ pkey,
    uint32_t* __restrict__ pid) {
    __shared__ uint32_t s_tmp[kEmitBlock / kWave];
    __shared__ uint32_t s_key[4 * kChunk];
    __shared__ uint32_t s_id[4 * kChunk];
    const int64_t live = live_points(n_live, n_vp);
    const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kEmitItems;
    uint32_t vals[kEmitItems], anc[kEmitItems];
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < kEmitItems; ++i) {
        const bool in = base + i < live;
        vals[i] = in ? zval[base + i] : 0u;
        anc[i] = in ? zanc[base + i] : 0u;
        cnt += __popc(vals[i] >> 28);
    }
    uint32_t total;
    uint32_t pos = block_excl_sum<kEmitBlock>(cnt, total, s_tmp);
    int64_t pix0 = 0, W0 = 0;
    if (n_views == 1) {
        pix0 = views[0].pixel_offset;
        W0 = views[0].W;
    }
#pragma unroll
    for (int i = 0; i < kEmitItems; ++i) {
        const uint32_t mask = vals[i] >> 28;
        if (mask == 0u) continue;
        const uint32_t vp = vals[i] & kVpMask;
        int64_t pix = pix0, W = W0;
        if (n_views != 1) {
            const GpuView& V = views[find_view(views, n_views, (int64_t)vp,
                                               [](const GpuView& g) { return g.vpoint_offset; })];
            pix = V.pixel_offset;
            W = V.W;
        }
        const int x0 = anc_x0(anc[i]), y0 = anc_y0(anc[i]);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!((mask >> c) & 1u)) continue;
            const int64_t q = pix + (int64_t)(y0 + (c >> 1)) * W + (x0 + (c & 1));
            s_key[pos] = (uint32_t)q;
            s_id[pos] = 4u * vp + (uint32_t)c;
            ++pos;
        }
    }
    __syncthreads();
    const uint32_t off = chunk_off[blockIdx.x];
    for (uint32_t j = threadIdx.x; j < total; j += kEmitBlock) {
        pkey[off + j] = s_key[j];
        pid[off + j] = s_id[j];
    }
}

void launch_emit(const uint32_t* zval_sorted, const uint32_t* n_live, const uint32_t* anc_sorted, const GpuView* views,
                 int n_views, int64_t n_vp, uint32_t* chunk_cnt, uint32_t* m_dev, uint32_t* pkey,
                 uint32_t* pid, uint32_t* clear, size_t clear_words, hipStream_t s) {
    const size_t chunks = emit_chunks(n_vp);
    if (chunks == 0) {
        launch_fill_u32(m_dev, 0u, 2, s);
        launch_fill_u32(clear, 0u, clear_words, s);
        return;
    }
    hipLaunchKernelGGL(k_emit_count<false>, dim3((unsigned)chunks), dim3(kEmitBlock), 0, s, zval_sorted,
                       n_vp, n_live, chunk_cnt, clear, clear_words);
    hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(1024), 0, s, chunk_cnt, chunks, m_dev, 0u);
    hipLaunchKernelGGL(k_emit_write, dim3((unsigned)chunks), dim3(kEmitBlock), 0, s, zval_sorted,
                       anc_sorted, views, n_views, n_vp, n_live, chunk_cnt, pkey, pid);
}

// Tile entries: one (tile, view point) pair per distinct square tile of
// 2^lg pixels a side (8x8 by default, 16x16 as a tuning) that the point's
// splats touch, written in the order of the depth-sorted points
// (tiles of one point in ascending corner order of first appearance).
__global__ __launch_bounds__(kEmitBlock) void k_tile_emit_write(
    const uint32_t* __restrict__ zval, const uint32_t* __restrict__ zanc,
    const GpuView* __restrict__ views, int n_views, int64_t n_vp, const uint32_t* __restrict__ n_live, int lg,
    const uint32_t* __restrict__ chunk_off, uint32_t* __restrict__ tkey,
    uint32_t* __restrict__ tval) {
    __shared__ uint32_t s_tmp[kEmitBlock / kWave];
    __shared__ uint32_t s_key[4 * kChunk];
    __shared__ uint32_t s_id[4 * kChunk];
    // A batch's depth-sorted points come from every view, so each item looks
    // its view up: for up to kLdsViews views in a copy of their tile
    // placement in LDS (read after the scan's barriers), which waits far less
    // than a search through memory.
    __shared__ int64_t s_vstart[kLdsViews], s_toff[kLdsViews], s_tpr[kLdsViews];
    const bool lds_views = n_views > 1 && n_views <= kLdsViews;
    if (lds_views) {
        for (int i = threadIdx.x; i < n_views; i += kEmitBlock) {
            s_vstart[i] = views[i].vpoint_offset;
            s_toff[i] = views[i].tile_offset;
            s_tpr[i] = views[i].tiles_x;
        }
    }
    const int64_t live = live_points(n_live, n_vp);
    const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kEmitItems;
    uint32_t vals[kEmitItems], anc[kEmitItems];
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < kEmitItems; ++i) {
        const bool in = base + i < live;
        vals[i] = in ? zval[base + i] : 0u;
        anc[i] = in ? zanc[base + i] : 0u;
        cnt += vals[i] >> 28;
    }
    uint32_t total;
    uint32_t pos = block_excl_sum<kEmitBlock>(cnt, total, s_tmp);
    // each item's tile placement is read once (for one view, once per thread)
    int64_t toff0 = 0, tpr0 = 0;
    if (n_views == 1) {
        toff0 = views[0].tile_offset;
        tpr0 = views[0].tiles_x;
    }
#pragma unroll
    for (int i = 0; i < kEmitItems; ++i) {
        if ((vals[i] >> 28) == 0u) continue;
        const uint32_t vp = vals[i] & kVpMask;
        int64_t toff = toff0, tpr = tpr0;
        if (lds_views) {
            int lo = 0, hi = n_views - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_vstart[mid] <= (int64_t)vp) lo = mid; else hi = mid - 1;
            }
            toff = s_toff[lo];
            tpr = s_tpr[lo];
        } else if (n_views != 1) {
            const GpuView& V = views[find_view(views, n_views, (int64_t)vp,
                                               [](const GpuView& g) { return g.vpoint_offset; })];
            toff = V.tile_offset;
            tpr = V.tiles_x;
        }
        const int x0 = anc_x0(anc[i]), y0 = anc_y0(anc[i]);
        const uint32_t mask = anc_mask(anc[i]);
        uint32_t seen[4];
        int n = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (!((mask >> c) & 1u)) continue;
            const int tx = (x0 + (c & 1)) >> lg, ty = (y0 + (c >> 1)) >> lg;
            const uint32_t t = (uint32_t)(toff + (int64_t)ty * tpr + tx);
            bool dup = false;
#pragma unroll
            for (int j = 0; j < 4; ++j) dup |= (j < n) && seen[j] == t;
            if (dup) continue;
            seen[n++] = t;
            s_key[pos] = t;
            s_id[pos] = vp;
            ++pos;
        }
    }
    __syncthreads();
    const uint32_t off = chunk_off[blockIdx.x];
    for (uint32_t j = threadIdx.x; j < total; j += kEmitBlock) {
        tkey[off + j] = s_key[j];
        tval[off + j] = s_id[j];
    }
}

void launch_tile_emit(const uint32_t* zval_sorted, const uint32_t* n_live, const uint32_t* anc_sorted, const GpuView* views,
                      int n_views, int64_t n_vp, int tile_log2, uint32_t* chunk_cnt, uint32_t* m_dev,
                      uint32_t* tkey, uint32_t* tval, uint32_t layout, uint32_t* clear, size_t clear_words,
                      hipStream_t s) {
    const size_t chunks = emit_chunks(n_vp);
    if (chunks == 0) {
        launch_fill_u32(m_dev, 0u, 1, s);
        launch_fill_u32(m_dev + 1, layout, 1, s);
        launch_fill_u32(clear, 0u, clear_words, s);
        return;
    }
    hipLaunchKernelGGL(k_emit_count<true>, dim3((unsigned)chunks), dim3(kEmitBlock), 0, s, zval_sorted,
                       n_vp, n_live, chunk_cnt, clear, clear_words);
    hipLaunchKernelGGL(k_scan_chunks, dim3(1), dim3(1024), 0, s, chunk_cnt, chunks, m_dev, layout);
    hipLaunchKernelGGL(k_tile_emit_write, dim3((unsigned)chunks), dim3(kEmitBlock), 0, s, zval_sorted,
                       anc_sorted, views, n_views, n_vp, n_live, tile_log2, chunk_cnt, tkey, tval);
}

}  // namespace inpc
