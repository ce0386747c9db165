// Host-side interface between the C ABI (api.cpp) and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace inpc {

// One entry of the tuning table: radix digit widths of the two sorts, keys
// per sort tile (BLOCK * items) and blend tile shape.
struct Tuning {
    int zdigit;       // digit bits of the per-point depth sort (0: from the key width)
    int pdigit;       // digit bits of the per-fragment pixel sort (0: from the key width)
    int sort_items;   // keys per thread in a sort tile (tile = 512 * items)
    int blend_shape;  // forward blend: lanes per pixel and wave tile, see blend_shape_dims()
    int bwd_shape;    // backward blend shape
    const char* name;
};

int tuning_count();
int auto_digit(int key_bits);
const Tuning& tuning(int id);

// -------------------------------------------------------------- profiling
// Optional per-stage timing with HIP events on the launch stream (off by
// default; see inpc_profile_begin/inpc_profile_end).  Stages may nest.
enum Stage {
    kStProject, kStDepthSort, kStEmit, kStPixelSort, kStRanges, kStBlendFwd, kStClearRecords,
    kStBlendBwd, kStPointReduce, kStSortUpsweep, kStSortScan, kStSortDownsweep, kStViewGrads,
    kStBlendWeight, kStMeanPlanes, kStAppearanceFwd, kStAppearanceBwd, kStSampleWeights, kStSampleDraw,
    kStProbUpdate, kNumStages
};
const char* stage_name(int stage);
void prof_begin(int stage, hipStream_t s);
void prof_end(int stage, hipStream_t s);

struct ProfScope {
    int st;
    hipStream_t s;
    ProfScope(int stage, hipStream_t stream) : st(stage), s(stream) { prof_begin(st, s); }
    ~ProfScope() { prof_end(st, s); }
};

// ------------------------------------------------------------------ launchers
void launch_upload_views(const GpuView* host_views, int n, GpuView* dev, hipStream_t s);

void launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t s);

// zval = vp | hb << 28 with hb the corner mask, or (tile_log2 > 0) the
// number of 2^tile_log2-pixel square tiles the point's splats touch.
// zanc = the record's anchor word (its own array, so that the depth sort can
// carry it to the emission).  payload (may be null): per view point, the
// record followed by the feature row (stored type), ps bytes per point,
// written for points with splats.
void launch_project(const float* xyz, const float* opa, const GpuView* views, int n_views,
                    int64_t n_vp, uint32_t zbase, uint32_t zkey_none, PointRec* rec, uint32_t* zkey,
                    uint32_t* zval, uint32_t* zanc, int tile_log2, const void* feat, int feat_row_bytes,
                    unsigned char* payload, int ps, hipStream_t s);

// Bytes per view point of the record + feature payload (64-byte multiple, so
// that a point's payload spans as few cache lines as possible).
inline int payload_stride(int F, int feat_dtype) {
    const int b = 16 + F * (feat_dtype == 1 ? 2 : 4);
    return (b + 63) / 64 * 64;
}

// Emission of the fragments of depth-sorted view points (count, scan, write).
constexpr int kEmitBlock = 256;
constexpr int kEmitItems = 4;
size_t emit_chunks(int64_t n_vp);
// m_dev[0] receives the fragment count M, m_dev[1] the layout code (0 here,
// the tile shape for tile entries); the count kernel also clears
// clear_words words at clear (the range array of the later ranges kernel).
// n_live: device count of the sorted view points to read (nullptr: n_vp);
// anc_sorted: their anchor words, in the same order.
void launch_emit(const uint32_t* zval_sorted, const uint32_t* n_live, const uint32_t* anc_sorted, const GpuView* views,
                 int n_views, int64_t n_vp, uint32_t* chunk_cnt, uint32_t* m_dev,
                 uint32_t* pkey, uint32_t* pid, uint32_t* clear, size_t clear_words, hipStream_t s);
// Tile entries of depth-sorted view points: (global tile id, view point).
void launch_tile_emit(const uint32_t* zval_sorted, const uint32_t* n_live, const uint32_t* anc_sorted, const GpuView* views,
                      int n_views, int64_t n_vp, int tile_log2, uint32_t* chunk_cnt, uint32_t* m_dev,
                      uint32_t* tkey, uint32_t* tval, uint32_t layout, uint32_t* clear, size_t clear_words,
                      hipStream_t s);

// Stable LSD radix sort of (u32 key, u32 value) pairs over key bits
// [0, bits).  n_dev (may be null) holds the live element count on the
// device; n_bound bounds it and sizes the grid.  Pass 0 reads (kin, vin) and
// writes (ka, va); later passes alternate between (ka, va) and (kb, vb), so
// the result is in (ka, va) after an odd number of passes (radix_passes)
// and in (kb, vb) after an even number (in (kin, vin) after none).
// (kin, vin) may alias (kb, vb).  counts holds sort_counts_words() words.
size_t sort_counts_words(int digit, int items, int64_t n_bound);
// live_out != nullptr: the first pass leaves out the keys equal to drop_key
// and writes how many it kept to *live_out; the later passes and the result
// hold only those (the result is *live_out keys long).  ain != nullptr: a
// second value per key, permuted with the pairs through aa / ab the way the
// values go through va / vb (three distinct arrays); required with live_out.
void launch_radix_sort(int digit, int items, int bits, const uint32_t* kin, const uint32_t* vin,
                       uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb,
                       const uint32_t* n_dev, int64_t n_bound, uint32_t* counts, hipStream_t s,
                       uint32_t drop_key = 0u, uint32_t* live_out = nullptr, const uint32_t* ain = nullptr,
                       uint32_t* aa = nullptr, uint32_t* ab = nullptr);
int radix_passes(int digit, int bits);
bool sort_valid(int digit, int items);

// Per-pixel [start, end) ranges of the pixel-sorted fragment keys.
// ``cleared``: the range array already holds zeros (cleared by the emission).
// order_tmp (may be null): the tile order's 66 counter words, cleared here.
void launch_ranges(const uint32_t* pkey_sorted, const uint32_t* m_dev, int64_t m_bound,
                   int64_t n_pixels, uint2* range, bool cleared, uint32_t* order_tmp, hipStream_t s);

// Tile dispatch order: perm[0, n_tiles) lists the tiles by descending entry
// count class (bit length of the count), so the blends start the heaviest
// tiles first.  order_tmp: the 66 counter words launch_ranges cleared.
void launch_tile_order(const uint2* range, int64_t n_tiles, uint32_t* order_tmp, uint32_t* perm, hipStream_t s);

// Per-pixel state kept from the forward blend for the backward.
struct alignas(16) PixelState {
    uint32_t n_blended;  // splats blended before termination
    uint32_t pad0, pad1, pad2;
};

void launch_blend_fwd(int F, int feat_dtype, int shape, const GpuView* views, int n_views,
                      int64_t n_tiles, const uint2* range, const uint32_t* ids, const PointRec* rec,
                      const void* feat, float tau, float* image, float* t_final, PixelState* state,
                      float* t_before, float* splat_weight, hipStream_t s);

// Octree sampling (Eq. 4) and probability updates (Eq. 2, Eq. 3).
struct SampleCam {
    float R[9], t[3];
    float fx, fy, cx, cy, near_p, far_p;
    int32_t W, H;
};
struct LevelTable {
    float f[32];   // 2^(l * lambda_l) rounded to float32, l = 0..31
};
void launch_sample_weights(const float* centre, const int32_t* level, const float* prob, int64_t n_leaves,
                           float root, float tau_d, const LevelTable& lt, const SampleCam& cam, bool view,
                           float* phat, uint32_t* max_bits, uint64_t* tile_sum, uint64_t* cdf, hipStream_t s);
// guide: 2^guide_bits(n_leaves) + 1 words of scratch (the inverse-CDF search's guide table).
int guide_bits(int64_t n_leaves);
void launch_sample_view(const float* centre, const int32_t* level, float root, const uint64_t* cdf,
                        int64_t n_leaves, uint32_t* guide, const SampleCam& cam, uint64_t seed0, uint64_t seed1,
                        int64_t n, int max_rounds, float* xyz, int32_t* leaf, unsigned long long* unresolved,
                        hipStream_t s);
void launch_sample_global(const float* centre, const int32_t* level, float root, const uint64_t* cdf,
                          int64_t n_leaves, uint32_t* guide, uint64_t seed0, uint64_t seed1, int64_t n,
                          uint32_t* counts, uint64_t* tile_sum, uint64_t* count_cdf, float* xyz, int32_t* leaf,
                          hipStream_t s);
void launch_prob_update(const int32_t* leaf, const float* b, int64_t n, int64_t n_leaves, float lambda_u,
                        float* prob, float* subdiv, uint32_t* kmax, uint32_t* kmin, hipStream_t s);

// Appearance step: opacity activation and degree-2 SH features per view
// point (forward), gradient of the raw rows per point (backward).
void launch_appearance_fwd(const float* xyz, const float* raw, const GpuView* views, int n_views,
                           int64_t n_vp, float* opa_out, void* feat_out, bool bf16, hipStream_t s);
void launch_appearance_bwd(const float* xyz, const float* raw, const GpuView* views, int n_views,
                           int64_t n_points, const float* g_opa, const float* g_feat, float* grad_raw,
                           hipStream_t s);

// Per-pixel average of K planes of ``plane`` floats each (float64 sums).
void launch_mean_planes(const float* in, int K, int64_t plane, float* out, hipStream_t s);

// Tile-list blend forward / backward (one block per tile, block b blending
// tile perm[b]).  t_ent holds, per
// sorted tile entry, T_k of the entry's four splats (by corner; zero where
// the splat is not blended in that tile).
void launch_tile_fwd(int F, int feat_dtype, int shape, const GpuView* views, int n_views, int64_t n_tiles,
                     const uint32_t* perm, const uint2* range, const uint32_t* vals, const unsigned char* payload, int ps,
                     float tau, float* image, float* t_final, PixelState* state, float4* t_ent,
                     float* splat_weight, hipStream_t s);
void launch_tile_bwd(int F, int feat_dtype, int shape, const GpuView* views, int n_views, int64_t n_tiles,
                     const uint32_t* perm, const uint2* range, const uint32_t* vals, const unsigned char* payload, int ps,
                     float tau, const PixelState* state, const float* g_img, const float* g_t,
                     float4* t_ent, int rebuild_t, float2* frec, hipStream_t s);

// Per-point blend weight from the per-splat weights T alpha (indexed by splat id).
void launch_blend_weight(int64_t n_vp, const PointRec* rec, const float* splat_weight, float* out,
                         hipStream_t s);

void launch_blend_bwd(int F, int feat_dtype, int shape, const GpuView* views, int n_views,
                      int64_t n_tiles, const uint2* range, const uint32_t* ids, const PointRec* rec,
                      const void* feat, float tau, const PixelState* state, const float* g_img,
                      const float* g_t, float* t_before, int rebuild_t, float2* frec, hipStream_t s);

void launch_point_reduce(int F, const GpuView* views, int n_views, int64_t n_vp,
                         const PointRec* rec, const float2* frec, const float* g_img,
                         float* grad_feat, float* grad_opa, float* blend_weight, hipStream_t s);

void launch_sum_view_grads(const GpuView* views, int n_views, int64_t n_points, int F,
                           const float* vg_feat, const float* vg_opa, float* g_feat, float* g_opa,
                           hipStream_t s);

// Blend shapes (must match dispatch_shape in blend_common.h): lanes per
// pixel L and wave-tile width WXP; a wave covers WXP x (64/L/WXP) pixels and
// a block of 4 waves a 2x2 arrangement of wave tiles.
struct BlendShape {
    int lanes, wxp;
};
inline BlendShape blend_shape_dims(int shape) {
    switch (shape) {
        case 1: return {2, 8};
        case 2: return {4, 4};
        case 3: return {8, 4};
        case 4: return {16, 2};
        default: return {1, 8};
    }
}
// Tile-list blending: one block per square tile of pixels with L lanes per
// pixel (shape 5: 16x16 tiles, 1 lane, 256 threads; shape 6: 8x8 tiles,
// 1 lane, 64 threads; shape 7: 8x8 tiles, 4 lanes, 256 threads; shape 8:
// 8x8 tiles, 2 lanes, 128 threads).
constexpr int kTileShape16 = 5;
constexpr int kTileShape8 = 6;
constexpr int kTileShape8x4 = 7;
constexpr int kTileShape8x2 = 8;
inline bool is_tile_shape(int shape) { return shape >= kTileShape16 && shape <= kTileShape8x2; }
inline int tile_size_of(int shape) { return shape == kTileShape16 ? 16 : 8; }
inline int tile_log2_of(int shape) { return shape == kTileShape16 ? 4 : 3; }

inline int blend_block_w(int shape) {
    return is_tile_shape(shape) ? tile_size_of(shape) : 2 * blend_shape_dims(shape).wxp;
}
inline int blend_block_h(int shape) {
    if (is_tile_shape(shape)) return tile_size_of(shape);
    const BlendShape b = blend_shape_dims(shape);
    return 2 * (64 / b.lanes / b.wxp);
}

}  // namespace inpc
