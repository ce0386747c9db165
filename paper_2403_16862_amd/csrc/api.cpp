// C ABI of the rasterizer: argument validation, buffer layout and the launch
// sequences of the forward (Algorithm 1) and backward (Appendix A.6) passes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/inpc_raster.h"
#include "internal.h"

namespace inpc {

// ------------------------------------------------------------ tuning table
// zdigit / pdigit = 0: choose the digit width from the key width (fewest
// passes of at most 9 bits, then the narrowest digit for that many passes).
static const Tuning kTunings[] = {
    {0, 0, 8, kTileShape8, kTileShape8, "auto digits, 4096-key tiles, tile-list blend 8x8 (entries per tile)"},
    {0, 0, 8, kTileShape8, kTileShape8x2, "auto digits, 4096-key tiles, tile-list blend 8x8, fwd 1 lane/pixel, bwd 2"},
    {0, 0, 8, kTileShape8x2, kTileShape8x2, "auto digits, 4096-key tiles, tile-list blend 8x8, 2 lanes/pixel"},
    {0, 0, 16, kTileShape8, kTileShape8, "auto digits, 8192-key tiles, tile-list blend 8x8 (entries per tile)"},
    {0, 0, 8, kTileShape16, kTileShape16, "auto digits, 4096-key tiles, tile-list blend 16x16 (entries per tile)"},
    {0, 0, 8, kTileShape8x4, kTileShape8x4, "auto digits, 4096-key tiles, tile-list blend 8x8, 4 lanes/pixel"},
    {0, 0, 8, kTileShape8x4, kTileShape8, "auto digits, 4096-key tiles, tile-list blend 8x8, fwd 4 lanes/pixel, bwd 1"},
    {0, 0, 8, 3, 4, "auto digits, 4096-key tiles, blend fwd 8 lanes/pixel 4x2, bwd 16 lanes/pixel 2x2"},
    {0, 0, 8, 3, 3, "auto digits, 4096-key tiles, blend fwd 8 lanes/pixel 4x2, bwd 8 lanes/pixel 4x2"},
    {0, 0, 8, 4, 4, "auto digits, 4096-key tiles, blend fwd 16 lanes/pixel 2x2, bwd 16 lanes/pixel 2x2"},
    {0, 0, 16, 3, 4, "auto digits, 8192-key tiles, blend fwd 8 lanes/pixel 4x2, bwd 16 lanes/pixel 2x2"},
    {8, 8, 8, 3, 4, "depth sort 8-bit, pixel sort 8-bit, 4096-key tiles, blend fwd 8, bwd 16 lanes/pixel"},
    {9, 11, 8, 3, 4, "depth sort 9-bit, pixel sort 11-bit, 4096-key tiles, blend fwd 8, bwd 16 lanes/pixel"},
    {0, 0, 8, 2, 2, "auto digits, 4096-key tiles, blend 4 lanes/pixel 4x4"},
    {0, 0, 8, 1, 1, "auto digits, 4096-key tiles, blend 2 lanes/pixel 8x4"},
    {0, 0, 8, 0, 0, "auto digits, 4096-key tiles, blend 1 lane/pixel 8x8"},
};

int auto_digit(int bits) {
    if (bits <= 0) return 8;
    const int passes = (bits + 8) / 9;
    const int d = (bits + passes - 1) / passes;
    return d < 7 ? 7 : d;
}

static int zdigit_of(const Tuning& t, int bits) { return t.zdigit ? t.zdigit : auto_digit(bits); }
static int pdigit_of(const Tuning& t, int bits) { return t.pdigit ? t.pdigit : auto_digit(bits); }
constexpr int kNumTunings = (int)(sizeof(kTunings) / sizeof(kTunings[0]));
constexpr int kDefaultTuning = 0;

// The backward may use its own blend shape, except in RECOMPUTE mode: there it
// rebuilds T_k with the forward's group recurrence, whose grouping must match.
static int bwd_shape_of(int tid, int mode) {
    return mode == INPC_RECOMPUTE ? kTunings[tid].blend_shape : kTunings[tid].bwd_shape;
}

int tuning_count() { return kNumTunings; }
const Tuning& tuning(int id) { return kTunings[id]; }

// --------------------------------------------------------------- errors
static thread_local char g_hip_msg[256] = "";

static int hip_fail(hipError_t e, const char* what) {
    std::snprintf(g_hip_msg, sizeof g_hip_msg, "%s: %s", what, hipGetErrorString(e));
    return INPC_EHIP;
}

static int check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return INPC_OK;
}

// ------------------------------------------------------------- problem
struct Problem {
    std::vector<GpuView> views;
    int64_t n_points = 0;   // length of the point arrays
    int64_t n_vp = 0;       // view points (sum of point counts)
    int64_t n_pixels = 0;   // packed pixels
    int64_t n_tiles = 0;    // blend tiles
    int F = 0, fdt = 0, mode = 0;
    int pixel_bits = 0;
    uint32_t zbase = 0;      // depth key = float bits of z - zbase
    uint32_t zkey_none = 0;  // depth key of points without splats (> every real key)
    int zbits = 32;          // key bits of the depth sort
    int tile_bits = 1;       // key bits of the tile sort at the blend shape's tile grid
    int tile_bits_max = 1;   // the same for the smallest tiles (sizes the sort scratch)
};

static bool finite_f(float x) { return std::isfinite(x); }

// A near plane of -0.0 keeps the same points as +0.0, but its bit pattern
// (0x80000000) would become the base of the depth keys and wrap them, so it
// is replaced by +0.0 before it is used anywhere.
static float canonical_near(float n) { return n == 0.0f ? 0.0f : n; }

static int check_camera(const inpc_camera_t& c) {
    if (c.width < 1 || c.height < 1) return INPC_EINVAL;
    if (c.width > 16383 || c.height > 16383) return INPC_EUNSUPPORTED;
    for (float x : c.R) if (!finite_f(x)) return INPC_EINVAL;
    for (float x : c.t) if (!finite_f(x)) return INPC_EINVAL;
    if (!finite_f(c.fx) || !finite_f(c.fy) || !finite_f(c.cx) || !finite_f(c.cy)) return INPC_EINVAL;
    if (!(c.near_plane >= 0.0f) || !(c.far_plane > c.near_plane) || std::isnan(c.far_plane))
        return INPC_EINVAL;
    return INPC_OK;
}

// Builds the problem description from a host view table; the blend shape
// decides the tile grid, so it is part of the problem.
static int make_problem(const inpc_view_t* views, int n_views, int64_t n_points, int F, int fdt,
                        int mode, int shape, Problem& pb, bool attr_per_vp = false) {
    if (!views || n_views < 1 || n_points < 0) return INPC_EINVAL;
    if (n_views > 65536) return INPC_EUNSUPPORTED;
    if (F < 1 || F > 64) return INPC_EUNSUPPORTED;
    if (fdt != INPC_F32 && fdt != INPC_BF16) return INPC_EINVAL;
    if (mode != INPC_SAVE && mode != INPC_RECOMPUTE) return INPC_EINVAL;
    pb = Problem{};
    pb.n_points = n_points;
    pb.F = F;
    pb.fdt = fdt;
    pb.mode = mode;
    const int bw = blend_block_w(shape), bh = blend_block_h(shape);
    int64_t vp = 0, pix = 0, tiles = 0;
    for (int v = 0; v < n_views; ++v) {
        const inpc_view_t& in = views[v];
        const int rc = check_camera(in.cam);
        if (rc) return rc;
        if (in.point_offset < 0 || in.point_count < 0 || in.point_offset > n_points ||
            in.point_count > n_points - in.point_offset)
            return INPC_EINVAL;
        if (in.pixel_offset != pix) return INPC_EINVAL;   // views are packed in order
        GpuView g{};
        std::memcpy(g.R, in.cam.R, sizeof g.R);
        std::memcpy(g.t, in.cam.t, sizeof g.t);
        g.fx = in.cam.fx; g.fy = in.cam.fy; g.cx = in.cam.cx; g.cy = in.cam.cy;
        g.near_p = canonical_near(in.cam.near_plane); g.far_p = in.cam.far_plane;
        g.W = in.cam.width; g.H = in.cam.height;
        g.point_offset = in.point_offset;
        g.vpoint_offset = vp;
        g.attr_offset = attr_per_vp ? vp : in.point_offset;
        g.point_count = in.point_count;
        g.pixel_offset = pix;
        g.tile_offset = tiles;
        g.tiles_x = (g.W + bw - 1) / bw;
        const int64_t tiles_y = (g.H + bh - 1) / bh;
        pb.views.push_back(g);
        vp += in.point_count;
        pix += (int64_t)g.W * g.H;
        tiles += g.tiles_x * tiles_y;
        if (vp >= ((int64_t)1 << 28)) return INPC_EOVERFLOW;
        if (pix >= (int64_t)0xFFFFFFFF) return INPC_EOVERFLOW;
    }
    if (tiles >= ((int64_t)1 << 31)) return INPC_EOVERFLOW;
    pb.n_vp = vp;
    pb.n_pixels = pix;
    pb.n_tiles = tiles;
    int64_t tiles8 = 0;
    for (const GpuView& g : pb.views) tiles8 += (int64_t)((g.W + 7) / 8) * ((g.H + 7) / 8);
    auto bits_for = [](int64_t n) {
        int b = 1;
        while (b < 32 && (((int64_t)1 << b) < n)) ++b;
        return b;
    };
    pb.tile_bits = bits_for(tiles);
    pb.tile_bits_max = bits_for(tiles8);
    int bits = 0;
    while (bits < 32 && (((int64_t)1 << bits) < pix)) ++bits;
    pb.pixel_bits = bits;
    // Depth keys: z lies strictly between a view's near and far planes, both
    // non-negative, where float bit patterns are monotone.
    uint32_t lo = 0xFFFFFFFFu, hi = 0;
    for (int v = 0; v < n_views; ++v) {
        uint32_t bn, bf;
        const float nc = canonical_near(views[v].cam.near_plane);
        std::memcpy(&bn, &nc, 4);
        std::memcpy(&bf, &views[v].cam.far_plane, 4);
        lo = std::min(lo, bn);
        hi = std::max(hi, bf);
    }
    pb.zbase = lo;
    pb.zkey_none = hi - lo;   // real keys are < bits(far) - zbase
    bits = 1;
    while (bits < 32 && (((uint64_t)1 << bits) <= pb.zkey_none)) ++bits;
    pb.zbits = bits;
    return INPC_OK;
}

// ------------------------------------------------------------- layout
struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

// Byte offsets of every buffer.  "fragment state" = point records, sorted
// splat ids and per-pixel ranges; it lives in ``saved`` in SAVE mode and in
// the workspace of whichever pass builds it in RECOMPUTE mode.
struct FragOffsets {
    size_t rec, ids, range, tk;   // tk: T_k of every blended splat (by sorted slot; tile lists: four per entry)
    size_t payload;               // record + feature row per view point (tile lists)
    size_t perm;                  // tile dispatch order, heaviest first (tile lists)
};
struct BuildOffsets {  // transient buffers of the fragment build
    size_t views, scalars, zk_in, zv_in, zk_a, zv_a, zk_b, zv_b, chunks, pk_a, pk_b, pv_other, counts;
    size_t order;   // tile-order class counters
};
struct Layout {
    size_t saved_bytes, fwd_bytes, bwd_bytes;
    size_t s_state, s_scalars;
    size_t s_views;             // SAVE mode: the device view table the backward reuses
    FragOffsets saved_frag;     // valid in SAVE mode (offsets into saved)
    FragOffsets fwd_frag;       // RECOMPUTE: offsets into fwd ws
    FragOffsets bwd_frag;       // RECOMPUTE: offsets into bwd ws
    BuildOffsets fwd_build, bwd_build;
    size_t b_views, b_frec;
};

static size_t max_counts_words(const Problem& pb) {
    size_t w = 0;
    for (int i = 0; i < kNumTunings; ++i) {
        const Tuning& t = kTunings[i];
        w = std::max(w, sort_counts_words(zdigit_of(t, pb.zbits), t.sort_items, pb.n_vp));
        w = std::max(w, sort_counts_words(pdigit_of(t, pb.pixel_bits), t.sort_items, 4 * pb.n_vp));
        w = std::max(w, sort_counts_words(pdigit_of(t, pb.tile_bits_max), t.sort_items, 4 * pb.n_vp));
        w = std::max(w, sort_counts_words(pdigit_of(t, pb.tile_bits_max - 1), t.sort_items, 4 * pb.n_vp));
    }
    return w;
}

// with_tk: room for the T_k of every blended splat; only a state the
// backward reads needs it (the RECOMPUTE forward keeps none).
static void carve_frag(Carver& c, const Problem& pb, FragOffsets& f, bool with_tk = true) {
    f.rec = c.take((size_t)pb.n_vp * sizeof(PointRec));
    f.ids = c.take((size_t)4 * pb.n_vp * 4);
    f.range = c.take((size_t)pb.n_pixels * sizeof(uint2));
    f.tk = with_tk ? c.take((size_t)4 * pb.n_vp * 16) : 0;   // at most 4 entries per point, 4 floats each
    f.payload = c.take((size_t)pb.n_vp * payload_stride(pb.F, pb.fdt));
    f.perm = c.take((size_t)pb.n_pixels * 4);   // tiles <= pixels
}

static void carve_build(Carver& c, const Problem& pb, BuildOffsets& b) {
    const size_t nv = (size_t)pb.n_vp, mb = 4 * nv;
    b.views = c.take(pb.views.size() * sizeof(GpuView));
    b.scalars = c.take(256);
    b.zk_in = c.take(nv * 4);
    b.zv_in = c.take(nv * 4);
    b.zk_a = c.take(nv * 4);
    b.zv_a = c.take(nv * 4);
    b.zk_b = c.take(nv * 4);
    b.zv_b = c.take(nv * 4);
    b.chunks = c.take((emit_chunks(pb.n_vp) + 1) * 4);
    b.pk_a = c.take(mb * 4);
    b.pk_b = c.take(mb * 4);
    b.pv_other = c.take(mb * 4);
    b.counts = c.take(max_counts_words(pb) * 4);
    b.order = c.take(512);   // tile-order counters (66 words)
}

static Layout make_layout(const Problem& pb) {
    Layout L{};
    Carver s, f, b;
    L.s_state = s.take((size_t)pb.n_pixels * sizeof(PixelState));
    L.s_scalars = s.take(256);
    if (pb.mode == INPC_SAVE) {
        L.s_views = s.take(pb.views.size() * sizeof(GpuView));
        carve_frag(s, pb, L.saved_frag);
    }
    carve_build(f, pb, L.fwd_build);
    if (pb.mode == INPC_RECOMPUTE) carve_frag(f, pb, L.fwd_frag, false);
    L.b_views = b.take(pb.views.size() * sizeof(GpuView));
    L.b_frec = b.take((size_t)4 * pb.n_vp * sizeof(float2));
    if (pb.mode == INPC_RECOMPUTE) {
        carve_build(b, pb, L.bwd_build);
        carve_frag(b, pb, L.bwd_frag);
    }
    L.saved_bytes = s.off;
    L.fwd_bytes = f.off;
    L.bwd_bytes = b.off;
    return L;
}

template <typename T>
static T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// ------------------------------------------------------------ profiling
static const char* kStageNames[kNumStages] = {
    "project", "depth_sort", "emit", "pixel_sort", "ranges", "blend_fwd", "clear_records",
    "blend_bwd", "point_reduce", "sort_upsweep", "sort_scan", "sort_downsweep", "view_grads",
    "blend_weight", "mean_planes", "appearance_fwd", "appearance_bwd", "sample_weights", "sample_draw",
    "prob_update"};

const char* stage_name(int st) { return (st >= 0 && st < kNumStages) ? kStageNames[st] : ""; }

static std::mutex g_prof_mu;
static bool g_prof_on = false;
struct ProfRec {
    int stage;
    hipEvent_t a, b;
};
static std::vector<hipEvent_t> g_prof_pool;
static size_t g_prof_used = 0;
static std::vector<std::pair<int, hipEvent_t>> g_prof_stack;
static std::vector<ProfRec> g_prof_recs;

static hipEvent_t prof_event() {
    if (g_prof_used == g_prof_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_prof_pool.push_back(e);
    }
    return g_prof_pool[g_prof_used++];
}

void prof_begin(int st, hipStream_t s) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    hipEvent_t e = prof_event();
    if (!e) return;
    (void)hipEventRecord(e, s);
    g_prof_stack.push_back({st, e});
}

void prof_end(int st, hipStream_t s) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (size_t i = g_prof_stack.size(); i-- > 0;) {
        if (g_prof_stack[i].first != st) continue;
        hipEvent_t e = prof_event();
        if (e) {
            (void)hipEventRecord(e, s);
            g_prof_recs.push_back({st, g_prof_stack[i].second, e});
        }
        g_prof_stack.erase(g_prof_stack.begin() + (long)i);
        return;
    }
}

// ------------------------------------------------------------ autotuner
static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune_cache;

static std::string bucket_key(const Problem& pb) {
    auto lg = [](int64_t x) {
        int b = 0;
        while (((int64_t)1 << b) < x) ++b;
        return b;
    };
    char buf[160];
    std::snprintf(buf, sizeof buf, "gfx950|V%d|N%d|P%d|F%d|T%d", (int)pb.views.size(), lg(pb.n_vp),
                  lg(pb.n_pixels), pb.F, pb.fdt);
    return buf;
}

static int resolve_tuning(int requested, const Problem& pb) {
    if (requested >= 0) return requested;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(bucket_key(pb));
    return it == g_tune_cache.end() ? kDefaultTuning : it->second;
}

// ------------------------------------------- tuning of each saved state
// The tuning id a forward used, keyed by its ``saved`` buffer.  The tuning
// fixes the layout of the fragment state (tile or per-pixel lists, tile
// size), so the backward must read the state with the forward's choice: a
// backward asked for tuning -1 takes the recorded id rather than the
// autotuner's cache (which may have changed in between), and one asked for
// another explicit id is rejected.  At most kSavedRecords buffers are
// remembered; the oldest record is dropped first.
static std::mutex g_saved_mu;
static std::map<const void*, std::pair<int, uint64_t>> g_saved_tuning;   // id, insertion stamp
static uint64_t g_saved_stamp = 0;
constexpr size_t kSavedRecords = 4096;

static void record_saved_tuning(const void* saved, int tid) {
    if (!saved) return;
    std::lock_guard<std::mutex> lk(g_saved_mu);
    g_saved_tuning[saved] = {tid, ++g_saved_stamp};
    if (g_saved_tuning.size() > kSavedRecords) {
        auto oldest = g_saved_tuning.begin();
        for (auto it = g_saved_tuning.begin(); it != g_saved_tuning.end(); ++it)
            if (it->second.second < oldest->second.second) oldest = it;
        g_saved_tuning.erase(oldest);
    }
}

static int saved_tuning(const void* saved) {
    if (!saved) return -1;
    std::lock_guard<std::mutex> lk(g_saved_mu);
    auto it = g_saved_tuning.find(saved);
    return it == g_saved_tuning.end() ? -1 : it->second.first;
}

// ------------------------------------------------- the fragment build
// Algorithm 1 up to the sorted, segmented splat list: projection and
// culling, depth sort of the points, order-preserving splat emission, global
// pixel sort, per-pixel ranges.  The depth digits of the (pixel, depth) key
// are sorted on the points (all splats of a point share its depth), so the
// splat-level sort only runs the pixel digits; together the passes form one
// stable LSD radix sort of the 64-bit (pixel << 32 | depth) keys.
// views: where the device view table goes (the saved state in SAVE mode, so
// that the backward reuses it).  m_dev[0] receives M, m_dev[1] the layout
// code of the lists (0: per-pixel lists, else the tile blend shape).
static void build_fragments(const Problem& pb, const Tuning& tn, const float* xyz,
                            const float* opacity, const void* feat, void* frag_base, const FragOffsets& fo,
                            void* build_base, const BuildOffsets& bo, GpuView* views, uint32_t* m_dev,
                            hipStream_t s) {
    const int nv = (int)pb.views.size();
    launch_upload_views(pb.views.data(), nv, views, s);
    PointRec* rec = at<PointRec>(frag_base, fo.rec);
    uint32_t* zk_in = at<uint32_t>(build_base, bo.zk_in);
    uint32_t* zv_in = at<uint32_t>(build_base, bo.zv_in);
    // The anchor words (in, and the two sort buffers) sit in the pixel sort's
    // first key buffer (4 n_vp words), which is unused until the emission
    // has read them.
    uint32_t* za_in = at<uint32_t>(build_base, bo.pk_a);
    uint32_t* za_a = za_in + pb.n_vp;
    uint32_t* za_b = za_a + pb.n_vp;
    const bool tile = is_tile_shape(tn.blend_shape);
    {
        ProfScope p(kStProject, s);
        launch_project(xyz, opacity, views, nv, pb.n_vp, pb.zbase, pb.zkey_none, rec, zk_in, zv_in, za_in,
                       tile ? tile_log2_of(tn.blend_shape) : 0, feat, pb.F * (pb.fdt == INPC_BF16 ? 2 : 4),
                       tile ? at<unsigned char>(frag_base, fo.payload) : nullptr, payload_stride(pb.F, pb.fdt),
                       s);
    }
    uint32_t* zk_a = at<uint32_t>(build_base, bo.zk_a);
    uint32_t* zv_a = at<uint32_t>(build_base, bo.zv_a);
    uint32_t* zk_b = at<uint32_t>(build_base, bo.zk_b);
    uint32_t* zv_b = at<uint32_t>(build_base, bo.zv_b);
    uint32_t* counts = at<uint32_t>(build_base, bo.counts);
    uint32_t* n_live = at<uint32_t>(build_base, bo.scalars) + 4;   // view points with splats, after the depth sort
    {
        ProfScope p(kStDepthSort, s);
        // points without splats (key zkey_none) leave the sort in its first pass
        launch_radix_sort(zdigit_of(tn, pb.zbits), tn.sort_items, pb.zbits, zk_in, zv_in, zk_a, zv_a, zk_b, zv_b,
                          nullptr, pb.n_vp, counts, s, pb.zkey_none, n_live, za_in, za_a, za_b);
    }
    const int zp = radix_passes(zdigit_of(tn, pb.zbits), pb.zbits);
    const uint32_t* zv_sorted = zp == 0 ? zv_in : ((zp & 1) ? zv_a : zv_b);
    const uint32_t* za_sorted = zp == 0 ? za_in : ((zp & 1) ? za_a : za_b);

    // Pixel sort (or tile sort of tile entries): emission writes (kb, vb);
    // the sorted values must end in the fragment-state id buffer.
    const int kbits = tile ? pb.tile_bits : pb.pixel_bits;
    const int pdig = pdigit_of(tn, kbits);
    const int pp = radix_passes(pdig, kbits);
    uint32_t* ids_final = at<uint32_t>(frag_base, fo.ids);
    uint32_t* pv_other = at<uint32_t>(build_base, bo.pv_other);
    uint32_t* pk_a = at<uint32_t>(build_base, bo.pk_a);
    uint32_t* pk_b = at<uint32_t>(build_base, bo.pk_b);
    uint32_t* pv_a = (pp & 1) ? ids_final : pv_other;
    uint32_t* pv_b = (pp & 1) ? pv_other : ids_final;
    {
        ProfScope p(kStEmit, s);
        uint32_t* range_words = reinterpret_cast<uint32_t*>(at<uint2>(frag_base, fo.range));
        const size_t n_range_words = (size_t)(tile ? pb.n_tiles : pb.n_pixels) * 2;
        if (tile)
            launch_tile_emit(zv_sorted, n_live, za_sorted, views, nv, pb.n_vp, tile_log2_of(tn.blend_shape),
                             at<uint32_t>(build_base, bo.chunks), m_dev, pk_b, pv_b, (uint32_t)tn.blend_shape,
                             range_words, n_range_words, s);
        else
            launch_emit(zv_sorted, n_live, za_sorted, views, nv, pb.n_vp, at<uint32_t>(build_base, bo.chunks), m_dev, pk_b,
                        pv_b, range_words, n_range_words, s);
    }
    {
        ProfScope p(kStPixelSort, s);
        launch_radix_sort(pdig, tn.sort_items, kbits, pk_b, pv_b, pk_a, pv_a, pk_b, pv_b,
                          m_dev, 4 * pb.n_vp, counts, s);
    }
    const uint32_t* pk_sorted = (pp & 1) ? pk_a : pk_b;
    {
        ProfScope p(kStRanges, s);
        launch_ranges(pk_sorted, m_dev, 4 * pb.n_vp, tile ? pb.n_tiles : pb.n_pixels,
                      at<uint2>(frag_base, fo.range), true, tile ? at<uint32_t>(build_base, bo.order) : nullptr, s);
        if (tile)
            launch_tile_order(at<uint2>(frag_base, fo.range), pb.n_tiles, at<uint32_t>(build_base, bo.order),
                              at<uint32_t>(frag_base, fo.perm), s);
    }
}

// ------------------------------------------------------------- logging
// INPC_LOG set (and not "0"): every rasterizing call reports on stderr the
// choices it made (tuning, list layout, sort digits and passes) or why it
// was rejected.  Read at each call, so it can be switched in a running process.
static bool log_on() {
    const char* e = std::getenv("INPC_LOG");
    return e && e[0] && std::strcmp(e, "0") != 0;
}

static void log_choices(const char* what, const Problem& pb, int tid, int shape) {
    if (!log_on()) return;
    const Tuning& tn = kTunings[tid];
    const bool tile = is_tile_shape(shape);
    const int kbits = tile ? pb.tile_bits : pb.pixel_bits;
    const int zd = zdigit_of(tn, pb.zbits), kd = pdigit_of(tn, kbits);
    std::fprintf(stderr,
                 "inpc: %s: %zu view(s), %lld view points, %lld pixels, F=%d %s, %s mode; tuning %d (%s); "
                 "depth sort %d bits = %d pass(es) of %d; %s sort %d bits = %d pass(es) of %d, %d-key tiles\n",
                 what, pb.views.size(), (long long)pb.n_vp, (long long)pb.n_pixels, pb.F,
                 pb.fdt == INPC_BF16 ? "bfloat16" : "float32", pb.mode == INPC_SAVE ? "save" : "recompute", tid,
                 tn.name, pb.zbits, radix_passes(zd, pb.zbits), zd, tile ? "tile" : "pixel", kbits,
                 radix_passes(kd, kbits), kd, 512 * tn.sort_items);
}

static int log_rejected(const char* what, int rc) {
    if (rc != INPC_OK && log_on()) std::fprintf(stderr, "inpc: %s rejected: %s\n", what, inpc_error_string(rc));
    return rc;
}

// ------------------------------------------------------------- forward
static int forward(const Problem& pb, int tid, const float* xyz, const void* feat,
                   const float* opacity, float tau, float* image, float* t_final, float* blend_weight,
                   void* saved, size_t saved_bytes, void* ws, size_t ws_bytes, hipStream_t s) {
    const Layout L = make_layout(pb);
    if (saved_bytes < L.saved_bytes || ws_bytes < L.fwd_bytes) return INPC_EWORKSPACE;
    if (pb.n_pixels > 0 && (!saved || !ws)) return INPC_EINVAL;
    const Tuning& tn = kTunings[tid];
    log_choices("forward", pb, tid, tn.blend_shape);
    uint32_t* m_dev = at<uint32_t>(saved, L.s_scalars);
    void* frag_base = pb.mode == INPC_SAVE ? saved : ws;
    const FragOffsets& fo = pb.mode == INPC_SAVE ? L.saved_frag : L.fwd_frag;
    GpuView* views = pb.mode == INPC_SAVE ? at<GpuView>(saved, L.s_views) : at<GpuView>(ws, L.fwd_build.views);
    build_fragments(pb, tn, xyz, opacity, feat, frag_base, fo, ws, L.fwd_build, views, m_dev, s);
    // Per-splat blend weights (indexed by splat id) reuse the pixel sort's
    // spare value buffer, which is dead once the sort has finished.
    float* splat_weight = blend_weight ? at<float>(ws, L.fwd_build.pv_other) : nullptr;
    if (splat_weight)
        launch_fill_u32(reinterpret_cast<uint32_t*>(splat_weight), 0u, (size_t)4 * pb.n_vp, s);
    {
        ProfScope p(kStBlendFwd, s);
        float* tk = pb.mode == INPC_SAVE ? at<float>(frag_base, fo.tk) : nullptr;
        if (is_tile_shape(tn.blend_shape))
            launch_tile_fwd(pb.F, pb.fdt, tn.blend_shape, views,
                            (int)pb.views.size(), pb.n_tiles, at<uint32_t>(frag_base, fo.perm),
                            at<uint2>(frag_base, fo.range), at<uint32_t>(frag_base, fo.ids),
                            at<unsigned char>(frag_base, fo.payload), payload_stride(pb.F, pb.fdt), tau, image, t_final,
                            at<PixelState>(saved, L.s_state), reinterpret_cast<float4*>(tk), splat_weight, s);
        else
            launch_blend_fwd(pb.F, pb.fdt, tn.blend_shape, views,
                             (int)pb.views.size(), pb.n_tiles, at<uint2>(frag_base, fo.range),
                             at<uint32_t>(frag_base, fo.ids), at<PointRec>(frag_base, fo.rec), feat, tau,
                             image, t_final, at<PixelState>(saved, L.s_state), tk, splat_weight, s);
    }
    if (blend_weight) {
        ProfScope p(kStBlendWeight, s);
        launch_blend_weight(pb.n_vp, at<PointRec>(frag_base, fo.rec), splat_weight, blend_weight, s);
    }
    return check_launch("inpc forward");
}

// ------------------------------------------------------------ backward
static int backward(const Problem& pb, int tid, float tau, const float* xyz, const void* feat,
                    const float* opacity, const void* saved, size_t saved_bytes,
                    const float* g_img, const float* g_t, float* grad_feat, float* grad_opa,
                    float* blend_weight, void* ws, size_t ws_bytes, hipStream_t s) {
    const Layout L = make_layout(pb);
    if (saved_bytes < L.saved_bytes || ws_bytes < L.bwd_bytes) return INPC_EWORKSPACE;
    if (pb.n_vp > 0 && (!saved || !ws)) return INPC_EINVAL;
    const Tuning& tn = kTunings[tid];
    void* sv = const_cast<void*>(saved);
    const void* frag_base;
    const FragOffsets* fo;
    const GpuView* views;
    const int bshape = bwd_shape_of(tid, pb.mode);
    log_choices("backward", pb, tid, bshape);
    if (pb.mode == INPC_SAVE) {
        // The forward left its device view table in the saved state; its tile
        // grid is the forward blend's, so a backward blend with other block
        // dimensions uploads its own table.
        if (blend_block_w(bshape) == blend_block_w(tn.blend_shape) &&
            blend_block_h(bshape) == blend_block_h(tn.blend_shape)) {
            views = at<GpuView>(sv, L.s_views);
        } else {
            launch_upload_views(pb.views.data(), (int)pb.views.size(), at<GpuView>(ws, L.b_views), s);
            views = at<GpuView>(ws, L.b_views);
        }
        frag_base = saved;
        fo = &L.saved_frag;
    } else {
        // Rebuild the fragment state exactly as the forward did.
        build_fragments(pb, tn, xyz, opacity, feat, ws, L.bwd_frag, ws, L.bwd_build,
                        at<GpuView>(ws, L.bwd_build.views), at<uint32_t>(ws, L.bwd_build.scalars), s);
        views = at<GpuView>(ws, L.bwd_build.views);
        frag_base = ws;
        fo = &L.bwd_frag;
    }
    float2* frec = at<float2>(ws, L.b_frec);
    {
        ProfScope p(kStClearRecords, s);
        launch_fill_u32(reinterpret_cast<uint32_t*>(frec), 0u, (size_t)8 * pb.n_vp, s);
    }
    {
    ProfScope p(kStBlendBwd, s);
    if (is_tile_shape(bshape))
        launch_tile_bwd(pb.F, pb.fdt, bshape, views, (int)pb.views.size(), pb.n_tiles,
                        at<const uint32_t>(const_cast<void*>(frag_base), fo->perm),
                        at<const uint2>(const_cast<void*>(frag_base), fo->range),
                        at<const uint32_t>(const_cast<void*>(frag_base), fo->ids),
                        at<const unsigned char>(const_cast<void*>(frag_base), fo->payload),
                        payload_stride(pb.F, pb.fdt), tau,
                        at<const PixelState>(sv, L.s_state), g_img, g_t,
                        at<float4>(const_cast<void*>(frag_base), fo->tk), pb.mode == INPC_RECOMPUTE ? 1 : 0,
                        frec, s);
    else
        launch_blend_bwd(pb.F, pb.fdt, bshape, views, (int)pb.views.size(), pb.n_tiles,
                         at<const uint2>(const_cast<void*>(frag_base), fo->range),
                         at<const uint32_t>(const_cast<void*>(frag_base), fo->ids),
                         at<const PointRec>(const_cast<void*>(frag_base), fo->rec), feat, tau,
                         at<const PixelState>(sv, L.s_state), g_img, g_t,
                         at<float>(const_cast<void*>(frag_base), fo->tk), pb.mode == INPC_RECOMPUTE ? 1 : 0,
                         frec, s);
    }
    ProfScope p(kStPointReduce, s);
    launch_point_reduce(pb.F, views, (int)pb.views.size(), pb.n_vp,
                        at<const PointRec>(const_cast<void*>(frag_base), fo->rec), frec, g_img,
                        grad_feat, grad_opa, blend_weight, s);
    return check_launch("inpc backward");
}

static bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

static int check_settings(const inpc_settings_t* st, int* tuning_req, float* tau, int* mode,
                          bool* attr_vp = nullptr) {
    if (!st) return INPC_EINVAL;
    if ((st->flags & ~INPC_ATTR_PER_VIEW_POINT) != 0) return INPC_EINVAL;
    if (attr_vp) *attr_vp = (st->flags & INPC_ATTR_PER_VIEW_POINT) != 0;
    if (!std::isfinite(st->t_threshold) || st->t_threshold < 0.0f) return INPC_EINVAL;
    if (st->tuning_id < -1 || st->tuning_id >= kNumTunings) return INPC_EINVAL;
    if (st->mode != INPC_SAVE && st->mode != INPC_RECOMPUTE) return INPC_EINVAL;
    *tuning_req = st->tuning_id;
    *tau = st->t_threshold;
    *mode = st->mode;
    return INPC_OK;
}

static int check_arrays(const Problem& pb, const float* xyz, const void* feat, const float* opa) {
    if (pb.n_points > 0 && (!xyz || !feat || !opa)) return INPC_EINVAL;
    if (pb.n_points > 0 && (!aligned(xyz, 4) || !aligned(opa, 4) || !aligned(feat, 16)))
        return INPC_EINVAL;
    return INPC_OK;
}

static inpc_view_t single_view(const inpc_camera_t* cam, int64_t n_points) {
    inpc_view_t v{};
    v.cam = *cam;
    v.point_offset = 0;
    v.point_count = n_points;
    v.pixel_offset = 0;
    return v;
}

static int shape_of(int tid) { return kTunings[tid].blend_shape; }

// Problem for sizing: tile counts do not enter any buffer size.
static int sizes_impl(const inpc_view_t* views, int n_views, int64_t n_points, int F, int fdt,
                      int mode, size_t* fwd_ws, size_t* saved, size_t* bwd_ws) {
    Problem pb;
    const int rc = make_problem(views, n_views, n_points, F, fdt, mode, 0, pb);
    if (rc) return rc;
    const Layout L = make_layout(pb);
    if (fwd_ws) *fwd_ws = L.fwd_bytes;
    if (saved) *saved = L.saved_bytes;
    if (bwd_ws) *bwd_ws = L.bwd_bytes;
    return INPC_OK;
}

static int fwd_checked(const float* xyz, const void* feat, int fdt, const float* opa, int64_t n_points,
                       int F, const inpc_view_t* views, int n_views, const inpc_settings_t* st,
                       float* image, float* t_final, float* blend_weight, void* saved, size_t saved_bytes,
                       void* ws, size_t ws_bytes, void* stream) {
    int treq, mode;
    float tau;
    bool avp;
    int rc = check_settings(st, &treq, &tau, &mode, &avp);
    if (rc) return rc;
    Problem pb;
    rc = make_problem(views, n_views, n_points, F, fdt, mode, 0, pb, avp);
    if (rc) return rc;
    const int tid = resolve_tuning(treq, pb);
    if (shape_of(tid) != 0) {
        rc = make_problem(views, n_views, n_points, F, fdt, mode, shape_of(tid), pb, avp);
        if (rc) return rc;
    }
    rc = check_arrays(pb, xyz, feat, opa);
    if (rc) return rc;
    if (!image || !t_final || !aligned(image, 16) || !aligned(t_final, 4)) return INPC_EINVAL;
    if (blend_weight && !aligned(blend_weight, 4)) return INPC_EINVAL;
    if ((saved && !aligned(saved, 256)) || (ws && !aligned(ws, 256))) return INPC_EINVAL;
    {
        const Layout L = make_layout(pb);
        if (saved_bytes < L.saved_bytes || ws_bytes < L.fwd_bytes) return INPC_EWORKSPACE;
        if (pb.n_pixels > 0 && (!saved || !ws)) return INPC_EINVAL;
    }
    record_saved_tuning(saved, tid);
    return forward(pb, tid, xyz, feat, opa, tau, image, t_final, blend_weight, saved, saved_bytes, ws,
                   ws_bytes, static_cast<hipStream_t>(stream));
}

static int fwd_impl(const float* xyz, const void* feat, int fdt, const float* opa, int64_t n_points,
                    int F, const inpc_view_t* views, int n_views, const inpc_settings_t* st,
                    float* image, float* t_final, float* blend_weight, void* saved, size_t saved_bytes,
                    void* ws, size_t ws_bytes, void* stream) {
    return log_rejected("forward", fwd_checked(xyz, feat, fdt, opa, n_points, F, views, n_views, st, image, t_final,
                                               blend_weight, saved, saved_bytes, ws, ws_bytes, stream));
}

// ------------------------------------------------------------ multisampling
// K point clouds sampled for one camera are rasterized as K views of that
// camera in one batched forward (no backward state is kept), then the K
// feature images and transmittances are averaged per pixel.
static int ms_views(const inpc_camera_t* cam, const int64_t* off, const int64_t* cnt, int K,
                    std::vector<inpc_view_t>& v) {
    if (!cam || !off || !cnt || K < 1) return INPC_EINVAL;
    if (K > 4096) return INPC_EUNSUPPORTED;
    const int64_t P = (int64_t)cam->width * cam->height;
    v.assign(K, inpc_view_t{});
    for (int k = 0; k < K; ++k) {
        v[k].cam = *cam;
        v[k].point_offset = off[k];
        v[k].point_count = cnt[k];
        v[k].pixel_offset = (int64_t)k * P;
    }
    return INPC_OK;
}

struct MsLayout {
    Layout L;
    size_t saved, fwd, img, tf, total;
};

static MsLayout ms_layout(const Problem& pb) {
    MsLayout m;
    m.L = make_layout(pb);
    Carver c;
    m.saved = c.take(m.L.saved_bytes);
    m.fwd = c.take(m.L.fwd_bytes);
    m.img = c.take((size_t)pb.n_pixels * pb.F * 4);
    m.tf = c.take((size_t)pb.n_pixels * 4);
    m.total = c.off;
    return m;
}

static int ms_impl(const float* xyz, const void* feat, int fdt, const float* opa, int64_t n_points, int F,
                   const inpc_camera_t* cam, const int64_t* off, const int64_t* cnt, int K,
                   const inpc_settings_t* st, float* image, float* t_final, void* ws, size_t ws_bytes,
                   size_t* ws_needed, void* stream) {
    std::vector<inpc_view_t> views;
    int rc = ms_views(cam, off, cnt, K, views);
    if (rc) return rc;
    int treq = -1, mode = INPC_RECOMPUTE;
    float tau = 1e-4f;
    bool avp = false;
    if (!ws_needed) {
        rc = check_settings(st, &treq, &tau, &mode, &avp);
        if (rc) return rc;
    }
    Problem pb;
    rc = make_problem(views.data(), K, n_points, F, fdt, INPC_RECOMPUTE, 0, pb, avp);
    if (rc) return rc;
    if (ws_needed) {
        *ws_needed = ms_layout(pb).total;
        return INPC_OK;
    }
    const int tid = resolve_tuning(treq, pb);
    if (shape_of(tid) != 0) {
        rc = make_problem(views.data(), K, n_points, F, fdt, INPC_RECOMPUTE, shape_of(tid), pb, avp);
        if (rc) return rc;
    }
    rc = check_arrays(pb, xyz, feat, opa);
    if (rc) return rc;
    if (!image || !t_final || !aligned(image, 16) || !aligned(t_final, 4)) return INPC_EINVAL;
    if (ws && !aligned(ws, 256)) return INPC_EINVAL;
    const MsLayout m = ms_layout(pb);
    if (ws_bytes < m.total) return INPC_EWORKSPACE;
    if (!ws) return INPC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* img_k = at<float>(ws, m.img);
    float* tf_k = at<float>(ws, m.tf);
    rc = forward(pb, tid, xyz, feat, opa, tau, img_k, tf_k, nullptr, at<void>(ws, m.saved), m.L.saved_bytes,
                 at<void>(ws, m.fwd), m.L.fwd_bytes, s);
    if (rc) return rc;
    const int64_t P = (int64_t)cam->width * cam->height;
    {
        ProfScope p(kStMeanPlanes, s);
        launch_mean_planes(img_k, K, P * F, image, s);
        launch_mean_planes(tf_k, K, P, t_final, s);
    }
    return check_launch("inpc multisample");
}

static int bwd_checked(const float* xyz, const void* feat, int fdt, const float* opa, int64_t n_points,
                       int F, const inpc_view_t* views, int n_views, const inpc_settings_t* st,
                       const void* saved, size_t saved_bytes, const float* g_img, const float* g_t,
                       float* grad_feat, float* grad_opa, float* blend_weight, void* ws, size_t ws_bytes,
                       void* stream) {
    int treq, mode;
    float tau;
    bool avp;
    int rc = check_settings(st, &treq, &tau, &mode, &avp);
    if (rc) return rc;
    Problem pb;
    rc = make_problem(views, n_views, n_points, F, fdt, mode, 0, pb, avp);
    if (rc) return rc;
    // The state must be read with the tuning of the forward that wrote it.
    const int rec = saved_tuning(saved);
    if (treq >= 0 && rec >= 0 && rec != treq) return INPC_EINVAL;
    const int tid = treq >= 0 ? treq : (rec >= 0 ? rec : resolve_tuning(-1, pb));
    if (bwd_shape_of(tid, mode) != 0) {
        rc = make_problem(views, n_views, n_points, F, fdt, mode, bwd_shape_of(tid, mode), pb, avp);
        if (rc) return rc;
    }
    rc = check_arrays(pb, xyz, feat, opa);
    if (rc) return rc;
    if (blend_weight && !aligned(blend_weight, 4)) return INPC_EINVAL;
    if (!g_img || !aligned(g_img, 16) || (g_t && !aligned(g_t, 4))) return INPC_EINVAL;
    if (pb.n_vp > 0 && (!grad_feat || !grad_opa || !aligned(grad_feat, 16) || !aligned(grad_opa, 4)))
        return INPC_EINVAL;
    if ((saved && !aligned(saved, 256)) || (ws && !aligned(ws, 256))) return INPC_EINVAL;
    return backward(pb, tid, tau, xyz, feat, opa, saved, saved_bytes, g_img, g_t, grad_feat, grad_opa,
                    blend_weight, ws, ws_bytes, static_cast<hipStream_t>(stream));
}

static int bwd_impl(const float* xyz, const void* feat, int fdt, const float* opa, int64_t n_points,
                    int F, const inpc_view_t* views, int n_views, const inpc_settings_t* st,
                    const void* saved, size_t saved_bytes, const float* g_img, const float* g_t,
                    float* grad_feat, float* grad_opa, float* blend_weight, void* ws, size_t ws_bytes,
                    void* stream) {
    return log_rejected("backward", bwd_checked(xyz, feat, fdt, opa, n_points, F, views, n_views, st, saved,
                                                saved_bytes, g_img, g_t, grad_feat, grad_opa, blend_weight, ws,
                                                ws_bytes, stream));
}

}  // namespace inpc

using namespace inpc;

// ------------------------------------------------ no-allocation forward
// The state and workspace of inpc_rasterize_fwd_noalloc: one array per GPU,
// held until the process ends.  In host code the name ``scratch`` only stands
// for the array; its device address on the current device comes from
// hipGetSymbolAddress (looked up once per device and kept), and only that
// address is handed to kernels.
constexpr size_t kScratchBytes = INPC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchDevices] = {};

static int scratch_of_current_device(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kScratchDevices) return INPC_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p || (reinterpret_cast<uintptr_t>(p) % 256) != 0) return INPC_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return INPC_OK;
}

extern "C" {

int inpc_version(void) { return 1; }

const char* inpc_error_string(int code) {
    switch (code) {
        case INPC_OK: return "ok";
        case INPC_EINVAL: return "invalid argument";
        case INPC_EWORKSPACE: return "workspace or saved buffer too small";
        case INPC_EUNSUPPORTED: return "unsupported feature count or image size";
        case INPC_EOVERFLOW: return "too many points or pixels for the index widths";
        case INPC_EHIP: return "HIP runtime error";
        case INPC_ESCRATCH: return "problem needs more than the fixed scratch of inpc_rasterize_fwd_noalloc";
        default: return "unknown error";
    }
}

const char* inpc_last_hip_error(void) { return g_hip_msg; }

int inpc_plain_sizes(int64_t n_points, const inpc_camera_t* cam, int32_t F, int32_t fdt,
                     int32_t mode, size_t* fwd_ws, size_t* saved, size_t* bwd_ws) {
    if (!cam) return INPC_EINVAL;
    const inpc_view_t v = single_view(cam, n_points);
    return sizes_impl(&v, 1, n_points, F, fdt, mode, fwd_ws, saved, bwd_ws);
}

int inpc_batched_sizes(const inpc_view_t* views, int32_t n_views, int64_t n_points, int32_t F,
                       int32_t fdt, int32_t mode, size_t* fwd_ws, size_t* saved, size_t* bwd_ws) {
    return sizes_impl(views, n_views, n_points, F, fdt, mode, fwd_ws, saved, bwd_ws);
}

int inpc_rasterize_fwd(const float* xyz, const void* feat, int32_t fdt, const float* opa,
                       int64_t n_points, int32_t F, const inpc_camera_t* cam,
                       const inpc_settings_t* st, float* image, float* t_final, float* blend_weight,
                       void* saved, size_t saved_bytes, void* ws, size_t ws_bytes, void* stream) {
    if (!cam) return INPC_EINVAL;
    const inpc_view_t v = single_view(cam, n_points);
    return fwd_impl(xyz, feat, fdt, opa, n_points, F, &v, 1, st, image, t_final, blend_weight, saved,
                    saved_bytes, ws, ws_bytes, stream);
}

int inpc_rasterize_bwd(const float* xyz, const void* feat, int32_t fdt, const float* opa,
                       int64_t n_points, int32_t F, const inpc_camera_t* cam,
                       const inpc_settings_t* st, const void* saved, size_t saved_bytes,
                       const float* g_img, const float* g_t, float* grad_feat, float* grad_opa,
                       float* blend_weight, void* ws, size_t ws_bytes, void* stream) {
    if (!cam) return INPC_EINVAL;
    const inpc_view_t v = single_view(cam, n_points);
    return bwd_impl(xyz, feat, fdt, opa, n_points, F, &v, 1, st, saved, saved_bytes, g_img, g_t,
                    grad_feat, grad_opa, blend_weight, ws, ws_bytes, stream);
}

int inpc_rasterize_fwd_noalloc(const float* xyz, const void* feat, int32_t fdt, const float* opa,
                               int64_t n_points, int32_t F, const inpc_camera_t* cam,
                               const inpc_settings_t* st, float* image, float* t_final, float* blend_weight,
                               void* stream) {
    if (!cam || !st) return INPC_EINVAL;
    if (st->mode != INPC_RECOMPUTE) return INPC_EINVAL;
    const inpc_view_t v = single_view(cam, n_points);
    size_t fws = 0, sv = 0;
    int rc = sizes_impl(&v, 1, n_points, F, fdt, INPC_RECOMPUTE, &fws, &sv, nullptr);
    if (rc) return rc;
    const size_t sv_room = (sv + 255) & ~(size_t)255;
    if (sv_room > kScratchBytes || fws > kScratchBytes - sv_room) return INPC_ESCRATCH;
    void* base = nullptr;
    rc = scratch_of_current_device(&base);
    if (rc) return rc;
    return fwd_impl(xyz, feat, fdt, opa, n_points, F, &v, 1, st, image, t_final, blend_weight, base, sv,
                    static_cast<unsigned char*>(base) + sv_room, fws, stream);
}

int inpc_rasterize_fwd_batched(const float* xyz, const void* feat, int32_t fdt, const float* opa,
                               int64_t n_points, int32_t F, const inpc_view_t* views,
                               int32_t n_views, const inpc_settings_t* st, float* image,
                               float* t_final, float* blend_weight, void* saved, size_t saved_bytes,
                               void* ws, size_t ws_bytes, void* stream) {
    return fwd_impl(xyz, feat, fdt, opa, n_points, F, views, n_views, st, image, t_final, blend_weight,
                    saved, saved_bytes, ws, ws_bytes, stream);
}

int inpc_rasterize_bwd_batched(const float* xyz, const void* feat, int32_t fdt, const float* opa,
                               int64_t n_points, int32_t F, const inpc_view_t* views,
                               int32_t n_views, const inpc_settings_t* st, const void* saved,
                               size_t saved_bytes, const float* g_img, const float* g_t,
                               float* grad_feat, float* grad_opa, float* blend_weight, void* ws,
                               size_t ws_bytes, void* stream) {
    return bwd_impl(xyz, feat, fdt, opa, n_points, F, views, n_views, st, saved, saved_bytes, g_img,
                    g_t, grad_feat, grad_opa, blend_weight, ws, ws_bytes, stream);
}

int inpc_sum_view_grads(const inpc_view_t* views, int32_t n_views, int64_t n_points, int32_t F,
                        const float* vg_feat, const float* vg_opa, float* g_feat, float* g_opa,
                        void* ws, size_t ws_bytes, void* stream) {
    Problem pb;
    int rc = make_problem(views, n_views, n_points, F, INPC_F32, INPC_SAVE, 0, pb);
    if (rc) return rc;
    if (n_points > 0 && (!g_feat || !g_opa || !aligned(g_feat, 16))) return INPC_EINVAL;
    if (pb.n_vp > 0 && (!vg_feat || !vg_opa || !aligned(vg_feat, 16))) return INPC_EINVAL;
    if (!ws || !aligned(ws, 256)) return INPC_EINVAL;
    static_assert(sizeof(GpuView) <= 256, "view table entry");
    if (ws_bytes < pb.views.size() * 256) return INPC_EWORKSPACE;
    if (n_points == 0) return INPC_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GpuView* dv = static_cast<GpuView*>(ws);
    launch_upload_views(pb.views.data(), (int)pb.views.size(), dv, s);
    launch_sum_view_grads(dv, (int)pb.views.size(), n_points, F, vg_feat, vg_opa, g_feat, g_opa, s);
    return check_launch("inpc_sum_view_grads");
}

static int appearance_views(const inpc_view_t* views, int n_views, int64_t n_points, void* ws,
                            size_t ws_bytes, Problem& pb) {
    const int rc = make_problem(views, n_views, n_points, 4, INPC_F32, INPC_SAVE, 0, pb);
    if (rc) return rc;
    if (!ws || !aligned(ws, 256)) return INPC_EINVAL;
    if (ws_bytes < pb.views.size() * 256) return INPC_EWORKSPACE;
    return INPC_OK;
}

int inpc_appearance_fwd(const float* xyz, const float* raw, int64_t n_points, const inpc_view_t* views,
                        int32_t n_views, float* opacity, void* feat, int32_t feat_dtype, void* ws,
                        size_t ws_bytes, void* stream) {
    Problem pb;
    int rc = appearance_views(views, n_views, n_points, ws, ws_bytes, pb);
    if (rc) return rc;
    if (feat_dtype != INPC_F32 && feat_dtype != INPC_BF16) return INPC_EINVAL;
    if (n_points > 0 && (!xyz || !raw || !aligned(xyz, 4) || !aligned(raw, 4))) return INPC_EINVAL;
    if (pb.n_vp > 0 && (!opacity || !feat || !aligned(opacity, 4) || !aligned(feat, 16))) return INPC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GpuView* dv = static_cast<GpuView*>(ws);
    launch_upload_views(pb.views.data(), (int)pb.views.size(), dv, s);
    {
        ProfScope p(kStAppearanceFwd, s);
        launch_appearance_fwd(xyz, raw, dv, (int)pb.views.size(), pb.n_vp, opacity, feat,
                              feat_dtype == INPC_BF16, s);
    }
    return check_launch("inpc_appearance_fwd");
}

int inpc_appearance_bwd(const float* xyz, const float* raw, int64_t n_points, const inpc_view_t* views,
                        int32_t n_views, const float* grad_opacity, const float* grad_feat, float* grad_raw,
                        void* ws, size_t ws_bytes, void* stream) {
    Problem pb;
    int rc = appearance_views(views, n_views, n_points, ws, ws_bytes, pb);
    if (rc) return rc;
    if (n_points > 0 && (!xyz || !raw || !grad_raw || !aligned(xyz, 4) || !aligned(raw, 4) ||
                         !aligned(grad_raw, 4)))
        return INPC_EINVAL;
    if (pb.n_vp > 0 && (!grad_opacity || !grad_feat || !aligned(grad_opacity, 4) || !aligned(grad_feat, 16)))
        return INPC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    GpuView* dv = static_cast<GpuView*>(ws);
    launch_upload_views(pb.views.data(), (int)pb.views.size(), dv, s);
    {
        ProfScope p(kStAppearanceBwd, s);
        launch_appearance_bwd(xyz, raw, dv, (int)pb.views.size(), n_points, grad_opacity, grad_feat, grad_raw,
                              s);
    }
    return check_launch("inpc_appearance_bwd");
}

// ------------------------------------------------------------ sampling
struct SampleLayout {
    size_t scalars, phat, cdf, tiles, counts, count_cdf, guide, total;
};

static SampleLayout sample_layout(int64_t n_leaves) {
    SampleLayout l;
    Carver c;
    const size_t L = (size_t)n_leaves, T = (L + 2047) / 2048 + 1;
    l.scalars = c.take(256);
    l.phat = c.take(4 * L);
    l.cdf = c.take(8 * L);
    l.tiles = c.take(8 * T);
    l.counts = c.take(4 * L);
    l.count_cdf = c.take(8 * L);
    l.guide = c.take(4 * (((size_t)1 << guide_bits(n_leaves)) + 1));
    l.total = c.off;
    return l;
}

static int check_octree(const float* centre, const int32_t* level, const float* prob, int64_t n_leaves,
                        float root_size, float lambda_l) {
    if (n_leaves < 1) return INPC_EINVAL;
    if (n_leaves > ((int64_t)1 << 24)) return INPC_EUNSUPPORTED;
    if (!centre || !level || !prob || !aligned(centre, 4) || !aligned(level, 4) || !aligned(prob, 4))
        return INPC_EINVAL;
    if (!std::isfinite(root_size) || !(root_size > 0.0f) || !std::isfinite(lambda_l)) return INPC_EINVAL;
    return INPC_OK;
}

static LevelTable level_table(float lambda_l) {
    LevelTable t;
    for (int l = 0; l < 32; ++l) t.f[l] = (float)std::pow(2.0, (double)l * (double)lambda_l);
    return t;
}

static SampleCam sample_cam(const inpc_camera_t& c) {
    SampleCam s;
    std::memcpy(s.R, c.R, sizeof s.R);
    std::memcpy(s.t, c.t, sizeof s.t);
    s.fx = c.fx; s.fy = c.fy; s.cx = c.cx; s.cy = c.cy;
    s.near_p = c.near_plane; s.far_p = c.far_plane;
    s.W = c.width; s.H = c.height;
    return s;
}

int inpc_multisample_sizes(int64_t n_points, const inpc_camera_t* cam, const int64_t* cloud_offset,
                           const int64_t* cloud_count, int32_t n_clouds, int32_t F, int32_t fdt,
                           size_t* ws_bytes) {
    if (!ws_bytes) return INPC_EINVAL;
    return ms_impl(nullptr, nullptr, fdt, nullptr, n_points, F, cam, cloud_offset, cloud_count, n_clouds,
                   nullptr, nullptr, nullptr, nullptr, 0, ws_bytes, nullptr);
}

int inpc_multisample_fwd(const float* xyz, const void* feat, int32_t fdt, const float* opa,
                         int64_t n_points, int32_t F, const inpc_camera_t* cam, const int64_t* cloud_offset,
                         const int64_t* cloud_count, int32_t n_clouds, const inpc_settings_t* st,
                         float* image, float* t_final, void* ws, size_t ws_bytes, void* stream) {
    return ms_impl(xyz, feat, fdt, opa, n_points, F, cam, cloud_offset, cloud_count, n_clouds, st, image,
                   t_final, ws, ws_bytes, nullptr, stream);
}

int inpc_sampling_sizes(int64_t n_leaves, size_t* ws_bytes) {
    if (!ws_bytes || n_leaves < 1) return INPC_EINVAL;
    if (n_leaves > ((int64_t)1 << 24)) return INPC_EUNSUPPORTED;
    *ws_bytes = sample_layout(n_leaves).total;
    return INPC_OK;
}

int inpc_sample_view(const float* centre, const int32_t* level, const float* prob, int64_t n_leaves,
                     float root_size, float lambda_l, float tau_d, const inpc_camera_t* cam, int64_t n_samples,
                     uint64_t seed0, uint64_t seed1, int32_t max_rounds, float* xyz, int32_t* leaf_index,
                     int64_t* n_unresolved, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_octree(centre, level, prob, n_leaves, root_size, lambda_l);
    if (rc) return rc;
    if (!cam) return INPC_EINVAL;
    rc = check_camera(*cam);
    if (rc) return rc;
    if (!std::isfinite(tau_d) || !(tau_d > 0.0f)) return INPC_EINVAL;
    if (n_samples < 0 || n_samples >= ((int64_t)1 << 31) || max_rounds < 0 || max_rounds > 65536)
        return INPC_EINVAL;
    if (!n_unresolved || !aligned(n_unresolved, 8)) return INPC_EINVAL;
    if (n_samples > 0 && (!xyz || !leaf_index || !aligned(xyz, 4) || !aligned(leaf_index, 4)))
        return INPC_EINVAL;
    if (!ws || !aligned(ws, 256)) return INPC_EINVAL;
    const SampleLayout l = sample_layout(n_leaves);
    if (ws_bytes < l.total) return INPC_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const SampleCam sc = sample_cam(*cam);
    {
        ProfScope p(kStSampleWeights, s);
        launch_sample_weights(centre, level, prob, n_leaves, root_size, tau_d, level_table(lambda_l), sc, true,
                              at<float>(ws, l.phat), at<uint32_t>(ws, l.scalars), at<uint64_t>(ws, l.tiles),
                              at<uint64_t>(ws, l.cdf), s);
    }
    {
        ProfScope p(kStSampleDraw, s);
        launch_sample_view(centre, level, root_size, at<uint64_t>(ws, l.cdf), n_leaves, at<uint32_t>(ws, l.guide), sc,
                           seed0, seed1,
                           n_samples, max_rounds, xyz, leaf_index,
                           reinterpret_cast<unsigned long long*>(n_unresolved), s);
    }
    return check_launch("inpc_sample_view");
}

int inpc_sample_global(const float* centre, const int32_t* level, const float* prob, int64_t n_leaves,
                       float root_size, float lambda_l, int64_t n_samples, uint64_t seed0, uint64_t seed1,
                       float* xyz, int32_t* leaf_index, void* ws, size_t ws_bytes, void* stream) {
    int rc = check_octree(centre, level, prob, n_leaves, root_size, lambda_l);
    if (rc) return rc;
    if (n_samples < 0 || n_samples >= ((int64_t)1 << 31)) return INPC_EINVAL;
    if (n_samples > 0 && (!xyz || !leaf_index || !aligned(xyz, 4) || !aligned(leaf_index, 4)))
        return INPC_EINVAL;
    if (!ws || !aligned(ws, 256)) return INPC_EINVAL;
    const SampleLayout l = sample_layout(n_leaves);
    if (ws_bytes < l.total) return INPC_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    inpc_camera_t dummy{};
    const SampleCam sc = sample_cam(dummy);
    {
        ProfScope p(kStSampleWeights, s);
        launch_sample_weights(centre, level, prob, n_leaves, root_size, 1.0f, level_table(lambda_l), sc, false,
                              at<float>(ws, l.phat), at<uint32_t>(ws, l.scalars), at<uint64_t>(ws, l.tiles),
                              at<uint64_t>(ws, l.cdf), s);
    }
    {
        ProfScope p(kStSampleDraw, s);
        launch_sample_global(centre, level, root_size, at<uint64_t>(ws, l.cdf), n_leaves, at<uint32_t>(ws, l.guide),
                             seed0, seed1,
                             n_samples, at<uint32_t>(ws, l.counts), at<uint64_t>(ws, l.tiles),
                             at<uint64_t>(ws, l.count_cdf), xyz, leaf_index, s);
    }
    return check_launch("inpc_sample_global");
}

int inpc_update_probabilities(const int32_t* leaf_index, const float* blend_weight, int64_t n_points,
                              int64_t n_leaves, float lambda_u, float* prob, float* subdiv, void* ws,
                              size_t ws_bytes, void* stream) {
    if (n_leaves < 1 || n_points < 0) return INPC_EINVAL;
    if (n_leaves > ((int64_t)1 << 24)) return INPC_EUNSUPPORTED;
    if (!std::isfinite(lambda_u)) return INPC_EINVAL;
    if (!prob || !subdiv || !aligned(prob, 4) || !aligned(subdiv, 4)) return INPC_EINVAL;
    if (n_points > 0 && (!leaf_index || !blend_weight || !aligned(leaf_index, 4) || !aligned(blend_weight, 4)))
        return INPC_EINVAL;
    if (!ws || !aligned(ws, 256)) return INPC_EINVAL;
    if (ws_bytes < sample_layout(n_leaves).total) return INPC_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver c;
    const size_t kmax = c.take(4 * (size_t)n_leaves), kmin = c.take(4 * (size_t)n_leaves);
    {
        ProfScope p(kStProbUpdate, s);
        launch_prob_update(leaf_index, blend_weight, n_points, n_leaves, lambda_u, prob, subdiv,
                           at<uint32_t>(ws, kmax), at<uint32_t>(ws, kmin), s);
    }
    return check_launch("inpc_update_probabilities");
}

int inpc_state_info(const inpc_view_t* views, int32_t n_views, int64_t n_points, int32_t F, int32_t fdt,
                    const void* saved, size_t saved_bytes, int64_t* stored_items, int32_t* layout,
                    void* stream) {
    Problem pb;
    int rc = make_problem(views, n_views, n_points, F, fdt, INPC_SAVE, 0, pb);
    if (rc) return rc;
    if (!saved || !stored_items || !layout) return INPC_EINVAL;
    const Layout L = make_layout(pb);
    if (saved_bytes < L.saved_bytes) return INPC_EWORKSPACE;
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "inpc_state_info sync");
    uint32_t sc[2] = {0, 0};
    e = hipMemcpy(sc, at<const uint32_t>(const_cast<void*>(saved), L.s_scalars), 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "inpc_state_info copy");
    *stored_items = sc[0];
    *layout = (int32_t)sc[1];
    return INPC_OK;
}

int inpc_tuning_count(void) { return kNumTunings; }

int inpc_saved_tuning(const void* saved) {
    const int id = saved_tuning(saved);
    return id >= 0 ? id : INPC_EINVAL;
}

const char* inpc_tuning_name(int32_t id) {
    if (id < 0 || id >= kNumTunings) return "";
    return kTunings[id].name;
}

int inpc_tuning_for(const inpc_view_t* views, int32_t n_views, int64_t n_points, int32_t F,
                    int32_t fdt) {
    Problem pb;
    const int rc = make_problem(views, n_views, n_points, F, fdt, INPC_SAVE, 0, pb);
    if (rc) return rc;
    return resolve_tuning(-1, pb);
}


int inpc_debug_fragments(const inpc_view_t* views, int32_t n_views, int64_t n_points, int32_t F,
                         int32_t fdt, const void* saved, size_t saved_bytes, const void* fwd_ws,
                         size_t fwd_ws_bytes, uint64_t* keys_host, uint32_t* ids_host, int64_t cap,
                         int64_t* m_out, uint32_t* n_blended_host, void* stream) {
    Problem pb;
    int rc = make_problem(views, n_views, n_points, F, fdt, INPC_SAVE, 0, pb);
    if (rc) return rc;
    if (!saved || !m_out) return INPC_EINVAL;
    const Layout L = make_layout(pb);
    if (saved_bytes < L.saved_bytes) return INPC_EWORKSPACE;
    if (keys_host && (!fwd_ws || fwd_ws_bytes < L.fwd_bytes)) return INPC_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "inpc_debug_fragments sync");
    uint32_t sc[2] = {0, 0};
    e = hipMemcpy(sc, at<const uint32_t>(const_cast<void*>(saved), L.s_scalars), 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "inpc_debug_fragments copy");
    const uint32_t m = sc[0];
    const bool tile = is_tile_shape((int)sc[1]);
    if (n_blended_host) {
        std::vector<PixelState> st((size_t)pb.n_pixels);
        e = hipMemcpy(st.data(), at<const PixelState>(const_cast<void*>(saved), L.s_state),
                      st.size() * sizeof(PixelState), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "inpc_debug_fragments copy");
        for (size_t q = 0; q < st.size(); ++q) n_blended_host[q] = st[q].n_blended;
    }
    auto copy = [&](void* dst, const void* src, size_t bytes) -> int {
        if (!bytes) return INPC_OK;
        const hipError_t err = hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost);
        return err == hipSuccess ? INPC_OK : hip_fail(err, "inpc_debug_fragments copy");
    };
    if (!tile) {
        *m_out = m;
        if (!keys_host || !ids_host || cap < (int64_t)m) return INPC_OK;
        std::vector<uint2> range((size_t)pb.n_pixels);
        std::vector<uint32_t> zk((size_t)pb.n_vp);
        if ((rc = copy(ids_host, at<const uint32_t>(const_cast<void*>(saved), L.saved_frag.ids), (size_t)m * 4)))
            return rc;
        if ((rc = copy(range.data(), at<const uint2>(const_cast<void*>(saved), L.saved_frag.range),
                       range.size() * sizeof(uint2))))
            return rc;
        if ((rc = copy(zk.data(), at<const uint32_t>(const_cast<void*>(fwd_ws), L.fwd_build.zk_in), zk.size() * 4)))
            return rc;
        // Keys from the device's own data: the pixel that owns each sorted slot
        // (from the per-pixel ranges) and the depth bits of the slot's point.
        for (int64_t q = 0; q < pb.n_pixels; ++q) {
            for (uint32_t i = range[q].x; i < range[q].y && i < m; ++i) {
                const uint32_t vp = ids_host[i] >> 2;
                const uint32_t zb = vp < zk.size() ? zk[vp] + pb.zbase : 0xFFFFFFFFu;
                keys_host[i] = ((uint64_t)q << 32) | zb;
            }
        }
        return INPC_OK;
    }
    // Tile lists: rebuild every pixel's splat list from the device's sorted
    // tile entries (entries of a tile restricted to one pixel keep their order).
    Problem pt;
    if ((rc = make_problem(views, n_views, n_points, F, fdt, INPC_SAVE, (int)sc[1], pt))) return rc;
    const int tsz = tile_size_of((int)sc[1]);
    if (!fwd_ws || fwd_ws_bytes < L.fwd_bytes) return INPC_EWORKSPACE;
    std::vector<uint32_t> ent(m);
    std::vector<uint2> range((size_t)pt.n_tiles);
    std::vector<PointRec> rec((size_t)pb.n_vp);
    std::vector<uint32_t> zk((size_t)pb.n_vp);
    if ((rc = copy(ent.data(), at<const uint32_t>(const_cast<void*>(saved), L.saved_frag.ids), (size_t)m * 4)))
        return rc;
    if ((rc = copy(range.data(), at<const uint2>(const_cast<void*>(saved), L.saved_frag.range),
                   range.size() * sizeof(uint2))))
        return rc;
    if ((rc = copy(rec.data(), at<const PointRec>(const_cast<void*>(saved), L.saved_frag.rec),
                   rec.size() * sizeof(PointRec))))
        return rc;
    if ((rc = copy(zk.data(), at<const uint32_t>(const_cast<void*>(fwd_ws), L.fwd_build.zk_in), zk.size() * 4)))
        return rc;
    std::vector<uint32_t> count((size_t)pb.n_pixels + 1, 0);
    auto for_each_splat = [&](auto&& emit) {
        size_t v = 0;
        for (int64_t t = 0; t < pt.n_tiles; ++t) {
            while (v + 1 < pt.views.size() && pt.views[v + 1].tile_offset <= t) ++v;
            const GpuView& V = pt.views[v];
            const int64_t lt = t - V.tile_offset;
            const int tx = (int)(lt % V.tiles_x), ty = (int)(lt / V.tiles_x);
            for (uint32_t i = range[t].x; i < range[t].y && i < m; ++i) {
                const uint32_t vp = ent[i];
                if (vp >= rec.size()) continue;
                const uint32_t a = rec[vp].anc;
                const int x0 = (int)(a & 0x3FFFu) - 1, y0 = (int)((a >> 14) & 0x3FFFu) - 1;
                for (int c = 0; c < 4; ++c) {
                    if (!((a >> (28 + c)) & 1u)) continue;
                    const int px = x0 + (c & 1), py = y0 + (c >> 1);
                    if (px / tsz != tx || py / tsz != ty) continue;
                    const int64_t q = V.pixel_offset + (int64_t)py * V.W + px;
                    emit(q, vp, c);
                }
            }
        }
    };
    for_each_splat([&](int64_t q, uint32_t, int) { ++count[(size_t)q + 1]; });
    for (size_t q = 0; q < (size_t)pb.n_pixels; ++q) count[q + 1] += count[q];
    const uint32_t total = count[(size_t)pb.n_pixels];
    *m_out = total;
    if (!keys_host || !ids_host || cap < (int64_t)total) return INPC_OK;
    for_each_splat([&](int64_t q, uint32_t vp, int c) {
        const uint32_t slot = count[(size_t)q]++;
        ids_host[slot] = 4u * vp + (uint32_t)c;
        keys_host[slot] = ((uint64_t)q << 32) | (zk[vp] + pb.zbase);
    });
    return INPC_OK;
}

// ------------------------------------------------------------- autotuner
static bool cache_merge_file(const char* path) {
    std::FILE* f = std::fopen(path, "r");
    if (!f) return false;
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
    std::fclose(f);
    size_t pos = 0;
    int loaded = 0;
    while ((pos = text.find('"', pos)) != std::string::npos) {
        const size_t end = text.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = text.substr(pos + 1, end - pos - 1);
        const size_t colon = text.find(':', end);
        if (colon == std::string::npos) break;
        int id = -1;
        if (std::sscanf(text.c_str() + colon + 1, "%d", &id) == 1 && id >= 0 && id < kNumTunings &&
            key.rfind("gfx950|", 0) == 0) {
            g_tune_cache[key] = id;
            ++loaded;
        }
        pos = colon + 1;
    }
    return loaded >= 0;
}

static bool cache_write_file(const char* path) {
    std::FILE* f = std::fopen(path, "w");
    if (!f) return false;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : g_tune_cache)
        std::fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < g_tune_cache.size() ? "," : "");
    std::fprintf(f, "}\n");
    std::fclose(f);
    return true;
}

int inpc_autotune_load(const char* path) {
    if (!path) return INPC_EINVAL;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const size_t before = g_tune_cache.size();
    if (!cache_merge_file(path)) return INPC_EINVAL;
    return (int)(g_tune_cache.size() - before);
}

int inpc_autotune(const float* xyz, const void* feat, int32_t fdt, const float* opa, int64_t n_points,
                  int32_t F, const inpc_view_t* views, int32_t n_views, float tau, float* image,
                  float* t_final, void* saved, size_t saved_bytes, const float* g_img,
                  float* grad_feat, float* grad_opa, void* ws, size_t ws_bytes, int32_t repeats,
                  const char* cache_path, float* best_ms, void* stream) {
    if (repeats < 1) repeats = 1;
    Problem pb;
    int rc = make_problem(views, n_views, n_points, F, fdt, INPC_SAVE, 0, pb);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return hip_fail(hipGetLastError(), "inpc_autotune events");
    int best = -1;
    float best_t = 0.0f;
    for (int tid = 0; tid < kNumTunings; ++tid) {
        inpc_settings_t st{tau, INPC_SAVE, tid, 0};
        auto step = [&]() -> int {
            int r = fwd_impl(xyz, feat, fdt, opa, n_points, F, views, n_views, &st, image, t_final, nullptr,
                             saved, saved_bytes, ws, ws_bytes, stream);
            if (r || !g_img) return r;
            return bwd_impl(xyz, feat, fdt, opa, n_points, F, views, n_views, &st, saved, saved_bytes,
                            g_img, nullptr, grad_feat, grad_opa, nullptr, ws, ws_bytes, stream);
        };
        rc = step();
        if (rc) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < repeats && rc == 0; ++r) rc = step();
        (void)hipEventRecord(e1, s);
        if (rc) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = hip_fail(hipGetLastError(), "inpc_autotune sync");
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)repeats;
        if (best < 0 || ms < best_t) {
            best = tid;
            best_t = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[bucket_key(pb)] = best;
        if (cache_path) {
            cache_merge_file(cache_path);
            g_tune_cache[bucket_key(pb)] = best;
            cache_write_file(cache_path);
        }
    }
    if (best_ms) *best_ms = best_t;
    return best;
}


int inpc_profile_stage_count(void) { return kNumStages; }

const char* inpc_profile_stage_name(int32_t stage) { return stage_name(stage); }

int inpc_profile_begin(void) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_recs.clear();
    g_prof_stack.clear();
    g_prof_used = 0;
    g_prof_on = true;
    return INPC_OK;
}

int inpc_profile_end(double* total_ms, int64_t* launches) {
    std::vector<ProfRec> recs;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_on = false;
        recs.swap(g_prof_recs);
        g_prof_stack.clear();
    }
    for (int i = 0; i < kNumStages; ++i) {
        if (total_ms) total_ms[i] = 0.0;
        if (launches) launches[i] = 0;
    }
    for (const ProfRec& r : recs) {
        const hipError_t e = hipEventSynchronize(r.b);
        if (e != hipSuccess) return hip_fail(e, "inpc_profile_end");
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        if (total_ms) total_ms[r.stage] += ms;
        if (launches) launches[r.stage] += 1;
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_used = 0;
    return INPC_OK;
}

}  // extern "C"
