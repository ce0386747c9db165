/*
 * inpc_raster.h -- C ABI of the MI355X (gfx950) differentiable bilinear point
 * rasterizer of INPC (Implicit Neural Point Clouds, arXiv 2403.16862).
 *
 * The operation (Appendix A.6, Algorithm 1, "Rasterize(C, P, A, F) -> I"):
 *   1. project every point with the camera (Section 3.4, Eq. 5) and cull it
 *      against the near/far planes and the image;
 *   2. splat it to the 2x2 pixels whose centres are closest to (u, v) with
 *      opacity alpha = alpha_h (1-|u-u_i|)(1-|v-v_i|) (Section 3.4, Eq. 6);
 *   3. order each pixel's splats by depth with one global sort: of
 *      (pixel, depth) keys, or (default) of (tile, depth) keys over one entry
 *      per (8x8 pixel tile, point) pair, whose order restricted to a pixel is
 *      that pixel's depth order;
 *   4. blend each pixel front to back, C = sum_i T_i alpha_i c_i,
 *      T_i = prod_{j<i} (1 - alpha_j) (Eq. 1), stopping after the splat that
 *      drops T below the threshold (Appendix A.6: 1e-4);
 *   5. backward: per-splat gradients in forward order, combined per point as
 *      a bilinear-weighted sum of its splat gradients (Appendix A.6).
 *
 * Conventions shared by every entry point
 *   - Pointers named *_host are host memory; every other array pointer is
 *     device memory on the current HIP device.  All device memory is owned by
 *     the caller; the library never allocates device memory in these calls.
 *   - Work is enqueued on ``stream`` (a hipStream_t; NULL = default stream)
 *     and the call returns without synchronising, so the calls can be
 *     captured in a HIP graph.  Outputs are valid once the stream reaches
 *     that point.
 *   - Arguments are validated on the host before anything is enqueued; on
 *     error nothing is enqueued and a negative INPC_E* code is returned.
 *     Per-element preconditions (opacity in [0,1], finite features) are not
 *     checked.
 *   - Environment: INPC_LOG set (and not "0") makes every rasterizing call
 *     print one line on stderr: the tuning, list layout and sort digits and
 *     passes it chose, or why it was rejected.  It is read at each call.
 *   - Layouts: xyz float32 [N,3] row-major; features [N,F] row-major in
 *     float32 or bfloat16 (``feat_dtype``); opacity float32 [N] (the activated
 *     alpha_h); image float32 [H,W,F]; t_final float32 [H,W] (the remaining
 *     transmittance, so alpha = 1 - t_final).  Gradients are always float32.
 *   - Camera: x_c = R x + t (R row-major), u = fx x_c/z_c + cx,
 *     v = fy y_c/z_c + cy; pixel (x,y) covers [x,x+1) x [y,y+1) and has its
 *     centre at (x+0.5, y+0.5).  A point is kept iff near < z_c < far and
 *     -1 < u < W+1, -1 < v < H+1.  Splats outside the image or with a zero
 *     bilinear factor are dropped and the rest are not renormalised.
 *     Equal depths in one pixel are ordered by ascending point index.
 *   - Limits: 1 <= F <= 64; 1 <= width, height <= 16383; total points over
 *     all views < 2^28; total pixels over all views < 2^32 - 1.
 *   - No gradient flows to positions or cameras (INPC samples positions
 *     rather than optimising them, Section 3.2).
 *   - The library keeps no state between calls except the autotuner's cache
 *     and, per ``saved`` buffer, the tuning id of the last forward that
 *     filled it (both guarded by a mutex); all entry points are reentrant.
 *   - A backward reads its state with the tuning of the forward that filled
 *     ``saved``: with settings.tuning_id = -1 it takes that recorded id (not
 *     the autotuner's current choice); an explicit id that differs from the
 *     recorded one is rejected with INPC_EINVAL.
 */
#ifndef INPC_RASTER_H
#define INPC_RASTER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define INPC_OK 0
#define INPC_EINVAL (-1)       /* null pointer, negative size, bad enum */
#define INPC_EWORKSPACE (-2)   /* a buffer is smaller than inpc_*_sizes() reports */
#define INPC_EUNSUPPORTED (-3) /* F outside 1..64, image side outside 1..16383 */
#define INPC_EOVERFLOW (-4)    /* too many points or pixels for the index widths */
#define INPC_EHIP (-5)         /* a HIP runtime call failed; see inpc_last_hip_error() */
#define INPC_ESCRATCH (-6)     /* needs more than INPC_NOALLOC_SCRATCH_BYTES (no-allocation call) */

typedef enum { INPC_F32 = 0, INPC_BF16 = 1 } inpc_dtype_t;

/* What the forward keeps for the backward (Appendix A.6 stores the sorted
 * key/index buffers; RECOMPUTE rebuilds them in the backward instead). */
typedef enum { INPC_SAVE = 0, INPC_RECOMPUTE = 1 } inpc_bwd_mode_t;

typedef struct {
    float R[9];           /* world -> camera rotation, row-major */
    float t[3];           /* world -> camera translation */
    float fx, fy, cx, cy; /* pinhole intrinsics in pixels */
    int32_t width, height;
    float near_plane, far_plane; /* the paper uses 0.01 and 100 (Appendix A.2) */
} inpc_camera_t;

typedef struct {
    float t_threshold; /* early-termination transmittance; 1e-4 in the paper; 0 disables */
    int32_t mode;      /* inpc_bwd_mode_t */
    int32_t tuning_id; /* -1: the autotuner's cached choice (else the default); >= 0: entry of the tuning table */
    int32_t flags;     /* 0 or INPC_ATTR_PER_VIEW_POINT */
} inpc_settings_t;

/* settings.flags: features and opacities are indexed by view point (row
 * sum_{u<v} point_count_u + i for point point_offset_v + i of view v) instead
 * of by point, so every view can carry its own view-dependent features (the
 * output of inpc_appearance_fwd).  Positions stay indexed by point. */
#define INPC_ATTR_PER_VIEW_POINT 1

/* One view of a batched call.  View v renders points
 * [point_offset, point_offset + point_count) of the point arrays (views may
 * share points) into pixels [pixel_offset, pixel_offset + W*H) of the packed
 * image [sum_v W_v H_v, F]. */
typedef struct {
    inpc_camera_t cam;
    int64_t point_offset;
    int64_t point_count;
    int64_t pixel_offset;
} inpc_view_t;

/* ---------------------------------------------------------------- sizes */

/* Bytes needed by the plain (one-view) calls for N points and this camera.
 * fwd_ws: forward workspace; saved: what the forward leaves for the backward
 * (depends on mode); bwd_ws: backward workspace.  Any output may be NULL. */
int inpc_plain_sizes(int64_t n_points, const inpc_camera_t *cam_host, int32_t F,
                     int32_t feat_dtype, int32_t mode, size_t *fwd_ws, size_t *saved,
                     size_t *bwd_ws);

/* Same for a batched call over n_views views (host table). */
int inpc_batched_sizes(const inpc_view_t *views_host, int32_t n_views, int64_t n_points,
                       int32_t F, int32_t feat_dtype, int32_t mode, size_t *fwd_ws,
                       size_t *saved, size_t *bwd_ws);

/* ------------------------------------------------------------ plain calls */

/* Forward rasterization of one view (Algorithm 1).
 * xyz [N,3] f32, feat [N,F] (feat_dtype), opacity [N] f32 in [0,1];
 * image [H,W,F] f32 and t_final [H,W] f32 are written in full.
 * blend_weight [N] f32 may be NULL (not computed).  Otherwise it is written
 * in full: per point, the blend weights T_k alpha_k (Eq. 1) of its blended
 * splats summed with the splats' bilinear weights as factors (the
 * bilinear combination of Appendix A.6), the per-point quantity that the
 * probability-field updates of Section 3.1 (Eq. 2, Eq. 3) consume; exact 0
 * for points without a blended splat.
 * saved (saved_bytes) receives the state the backward needs; ws is scratch. */
int inpc_rasterize_fwd(const float *xyz, const void *feat, int32_t feat_dtype,
                       const float *opacity, int64_t n_points, int32_t F,
                       const inpc_camera_t *cam_host, const inpc_settings_t *settings_host,
                       float *image, float *t_final, float *blend_weight, void *saved,
                       size_t saved_bytes, void *ws, size_t ws_bytes, void *stream);

/* Backward of inpc_rasterize_fwd for L with dL/dimage = grad_image [H,W,F]
 * and dL/dt_final = grad_t_final [H,W] (may be NULL = zero).  The inputs and
 * settings must be those of the forward that filled ``saved``.
 * Writes grad_feat [N,F] f32 and grad_opacity [N] f32 in full (points that
 * produce no blended splat get exact zeros).  Deterministic: no float
 * atomics; every gradient is summed in a fixed order.
 * blend_weight [N] f32 (may be NULL): the same per-point blend weight as the
 * forward's optional output, obtained here almost for free from the
 * per-splat records the backward already reduces (training computes the
 * probability updates after the backward). */
int inpc_rasterize_bwd(const float *xyz, const void *feat, int32_t feat_dtype,
                       const float *opacity, int64_t n_points, int32_t F,
                       const inpc_camera_t *cam_host, const inpc_settings_t *settings_host,
                       const void *saved, size_t saved_bytes, const float *grad_image,
                       const float *grad_t_final, float *grad_feat, float *grad_opacity,
                       float *blend_weight, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------- no-allocation forward */

/* Bytes of the fixed device scratch behind inpc_rasterize_fwd_noalloc: one
 * array of this size per GPU the library runs on, held until the process
 * ends. */
#define INPC_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward of inpc_rasterize_fwd with its state and workspace taken from a
 * file-scope device array of INPC_NOALLOC_SCRATCH_BYTES instead of caller
 * buffers.  Nothing is allocated, by the library or by any routine it calls.
 * Arguments and outputs as for inpc_rasterize_fwd; no state is kept for a
 * backward, so settings->mode must be INPC_RECOMPUTE (else INPC_EINVAL).
 * The results equal those of inpc_rasterize_fwd with the same arguments.
 * A problem whose recompute-mode state plus forward workspace
 * (inpc_plain_sizes with mode INPC_RECOMPUTE; each part rounded up to 256
 * bytes) exceeds INPC_NOALLOC_SCRATCH_BYTES is rejected with INPC_ESCRATCH
 * before anything is enqueued (up to about 1.37M points fit at 1280x720 with
 * F=8, 0.87M at 1920x1080 with F=16 float32, 1.19M with F=16 bfloat16).
 * Every call on one GPU uses that GPU's one array, whose contents the
 * previous call left there; every buffer that must start at a value is set
 * by the call's own kernels.  Calls that overlap on one GPU (other streams,
 * other threads) race on the array: serialise them.  The first call on each
 * device looks up the array's device address (a runtime query, no
 * allocation); make that first call outside graph capture. */
int inpc_rasterize_fwd_noalloc(const float *xyz, const void *feat, int32_t feat_dtype,
                               const float *opacity, int64_t n_points, int32_t F,
                               const inpc_camera_t *cam_host, const inpc_settings_t *settings_host,
                               float *image, float *t_final, float *blend_weight, void *stream);

/* ---------------------------------------------------------- batched calls */

/* Forward over several views of uneven size and point count in one launch
 * sequence: one projection, one global depth sort, one fragment emission,
 * one global pixel sort and one blend for all views.  This is the shape of
 * the paper's multisampled rendering (Section 3.2, viewpoint-specific
 * sampling: several clouds per frame; Table 2: 4 x 8M points per frame) and
 * of rendering several training views at once.  Packed outputs:
 * image [sum P_v, F], t_final [sum P_v], blend_weight (NULL or one entry per
 * view point, in view order) [sum point_count_v].  n_points is the length of the
 * point arrays.  The view table is read on the host and passed to the
 * kernels by value, so the call can be graph-captured. */
int inpc_rasterize_fwd_batched(const float *xyz, const void *feat, int32_t feat_dtype,
                               const float *opacity, int64_t n_points, int32_t F,
                               const inpc_view_t *views_host, int32_t n_views,
                               const inpc_settings_t *settings_host, float *image,
                               float *t_final, float *blend_weight, void *saved,
                               size_t saved_bytes, void *ws, size_t ws_bytes, void *stream);

/* Backward of the batched forward (per-splat gradients in forward order,
 * combined per point with the bilinear weights, Appendix A.6, for every view
 * of the batch; Section 3.2's multisampling shares points between views).
 * Gradients are per *view point*: row
 * (sum_{u<v} point_count_u) + i belongs to point point_offset_v + i of view
 * v, so grad_feat is [sum_v point_count_v, F] and grad_opacity
 * [sum_v point_count_v].  inpc_sum_view_grads() folds them onto the points. */
int inpc_rasterize_bwd_batched(const float *xyz, const void *feat, int32_t feat_dtype,
                               const float *opacity, int64_t n_points, int32_t F,
                               const inpc_view_t *views_host, int32_t n_views,
                               const inpc_settings_t *settings_host, const void *saved,
                               size_t saved_bytes, const float *grad_image,
                               const float *grad_t_final, float *grad_feat,
                               float *grad_opacity, float *blend_weight, void *ws,
                               size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ appearance */

/* Per-point appearance step (Section 3.3).  raw [N,37] f32 per point: the
 * opacity logit x, then 36 coefficients of real spherical harmonics of
 * degree 2 for 4 output channels, coefficient (basis j, channel c) at
 * 1 + 4j + c; basis order (l,m) = (0,0),(1,-1),(1,0),(1,1),(2,-2),(2,-1),
 * (2,0),(2,1),(2,2), the real harmonics being sqrt(2) Re / Im of the
 * complex ones with the Condon-Shortley phase.
 * Forward, per view point (views as in the batched calls; pixel offsets must
 * be packed): opacity [sum point_count] f32 = 1 - exp(-exp(x)), and the
 * 4-D feature [sum point_count, 4] (feat_dtype; bfloat16 rounded to nearest
 * even) = sum_j Y_j(d) coef[j][c], d the unit vector from the view's camera
 * centre -R^T t to the point (zero for a point at the centre).  These rows
 * feed the rasterizer with INPC_ATTR_PER_VIEW_POINT.
 * Backward: grad_raw [N,37] f32, written in full, = the sum over the views
 * containing each point (in view order) of the chain rule through both
 * parts; points in no view get zeros.  Positions get no gradient.
 * ws: at least 256 * n_views bytes of device scratch (the view table). */
int inpc_appearance_fwd(const float *xyz, const float *raw, int64_t n_points,
                        const inpc_view_t *views_host, int32_t n_views, float *opacity,
                        void *feat, int32_t feat_dtype, void *ws, size_t ws_bytes, void *stream);
int inpc_appearance_bwd(const float *xyz, const float *raw, int64_t n_points,
                        const inpc_view_t *views_host, int32_t n_views,
                        const float *grad_opacity, const float *grad_feat, float *grad_raw,
                        void *ws, size_t ws_bytes, void *stream);

/* -------------------------------------------------------- octree sampling */

/* Point sampling from the probability octree (Section 3.2, Eq. 4; Appendix
 * A.4) and the per-leaf probability updates (Section 3.1, Eq. 2, Eq. 3).
 * The octree is given by its leaves: centre [L,3] f32 (world), level [L]
 * int32 (0..31; edge = root_size * 2^-level), prob [L] f32 in [0,1].
 * 1 <= L <= 2^24 (the paper caps the octree at 256^3 leaves).
 *
 * Re-weighting (Eq. 4): p_hat = 1_visible * p / (d * 2^(level*lambda_l)),
 * d = max(|z_view(centre) - near| / far, tau_d) (Appendix A.4); a leaf is
 * visible unless its cube lies entirely outside one of the six frustum
 * half-spaces (near, far, u = 0, u = W, v = 0, v = H).  The global
 * extraction omits 1_visible and d.  All in float32, in a fixed order.
 * Multinomial sampling with replacement inverts the integer CDF of
 * w = floor(p_hat * 2^(38 - e)) (m = max p_hat < 2^e): the leaf of a 64-bit
 * random x is the first i with CDF_i > floor(x * W_total / 2^64).
 * Random numbers: Philox4x64-10 with key (seed0, seed1) and counter
 * (sample, round, stream, 0), stream 1 here (word 0: leaf, top 24 bits of
 * words 1..3: position fractions f), stream 2 for the global extraction.
 * Position = centre + (f - 0.5) * edge per axis (float32).
 *
 * inpc_sample_view: n_samples viewpoint-specific samples, xyz [n,3] f32 and
 * leaf_index [n] int32 in sample order.  A sample outside the image
 * frustum (not near < z < far, 0 <= u < W, 0 <= v < H) is drawn again with
 * the next round, at most max_rounds times (Appendix A.4); max_rounds = 0
 * keeps every first draw (inference with multisampling).  *n_unresolved
 * (device int64) receives the number of samples still outside after
 * max_rounds.  If no leaf is visible every sample is unresolved, with NaN
 * positions and leaf -1.
 * inpc_sample_global: viewpoint-independent extraction; the multinomial
 * draws give per-leaf counts, outputs are ordered by leaf, and the j-th
 * sample of a leaf sits at the 3D Halton point of index j+1 (bases 2, 3, 5)
 * inside the leaf.
 * inpc_update_probabilities: for each leaf with points (leaf_index[i] =
 * leaf; out-of-range indices are ignored), p = max(lambda_u * p, max b) and
 * q = max(lambda_u * q, max b - min b) over its points' blend weights b
 * (the per-point output of inpc_rasterize_fwd); leaves without points decay:
 * p = lambda_u * p, q = lambda_u * q.  prob and subdiv [L] are updated in
 * place.  Deterministic (integer atomics on order-preserving keys).
 * ws: inpc_sampling_sizes() bytes of device scratch, 256-byte aligned. */
int inpc_sampling_sizes(int64_t n_leaves, size_t *ws_bytes);
int inpc_sample_view(const float *centre, const int32_t *level, const float *prob, int64_t n_leaves,
                     float root_size, float lambda_l, float tau_d, const inpc_camera_t *cam_host,
                     int64_t n_samples, uint64_t seed0, uint64_t seed1, int32_t max_rounds,
                     float *xyz, int32_t *leaf_index, int64_t *n_unresolved, void *ws,
                     size_t ws_bytes, void *stream);
int inpc_sample_global(const float *centre, const int32_t *level, const float *prob,
                       int64_t n_leaves, float root_size, float lambda_l, int64_t n_samples,
                       uint64_t seed0, uint64_t seed1, float *xyz, int32_t *leaf_index, void *ws,
                       size_t ws_bytes, void *stream);
int inpc_update_probabilities(const int32_t *leaf_index, const float *blend_weight,
                              int64_t n_points, int64_t n_leaves, float lambda_u, float *prob,
                              float *subdiv, void *ws, size_t ws_bytes, void *stream);

/* --------------------------------------------------------- multisampling */

/* Multisampled inference (Section 3.2: for one viewpoint, several point
 * clouds are sampled and rasterized, and each pixel's features are
 * averaged).  Cloud k is the range [cloud_offset[k], +cloud_count[k]) of the
 * point arrays (host arrays; 1 <= n_clouds <= 4096; clouds may overlap).
 * image [H,W,F] f32 receives the per-pixel mean of the K feature images and
 * t_final [H,W] f32 the mean of the K final transmittances (compositing over
 * a background is linear, so the mean of composited images equals the mean
 * image composited with the mean transmittance).  Means are summed in f64
 * in cloud order.  Forward only; settings->mode is validated but no backward
 * state is kept.  ws: inpc_multisample_sizes() bytes, 256-byte aligned. */
int inpc_multisample_sizes(int64_t n_points, const inpc_camera_t *cam_host,
                           const int64_t *cloud_offset_host, const int64_t *cloud_count_host,
                           int32_t n_clouds, int32_t F, int32_t feat_dtype, size_t *ws_bytes);
int inpc_multisample_fwd(const float *xyz, const void *feat, int32_t feat_dtype,
                         const float *opacity, int64_t n_points, int32_t F,
                         const inpc_camera_t *cam_host, const int64_t *cloud_offset_host,
                         const int64_t *cloud_count_host, int32_t n_clouds,
                         const inpc_settings_t *settings_host, float *image, float *t_final,
                         void *ws, size_t ws_bytes, void *stream);

/* grad_feat[p] = sum over views v containing p, in view order, of the view
 * point rows of p (and likewise grad_opacity).  Points no view contains get
 * zeros.  Deterministic.  ws: at least 256 * n_views bytes of device scratch. */
int inpc_sum_view_grads(const inpc_view_t *views_host, int32_t n_views, int64_t n_points,
                        int32_t F, const float *view_grad_feat, const float *view_grad_opacity,
                        float *grad_feat, float *grad_opacity, void *ws, size_t ws_bytes,
                        void *stream);

/* What a forward stored (synchronises the stream): *stored_items = number of
 * list items (splats for per-pixel lists, tile entries for tile lists) and
 * *layout = 0 for per-pixel lists or the tile-list blend shape (5: 16x16
 * tiles; 6, 7, 8: 8x8 tiles with 1, 4 or 2 lanes per pixel).  Arguments as
 * for inpc_debug_fragments. */
int inpc_state_info(const inpc_view_t *views_host, int32_t n_views, int64_t n_points, int32_t F,
                    int32_t feat_dtype, const void *saved, size_t saved_bytes,
                    int64_t *stored_items, int32_t *layout, void *stream);

/* ----------------------------------------------------------- autotuning */

/* Number of entries of the tuning table and a printable description. */
int inpc_tuning_count(void);
const char *inpc_tuning_name(int32_t tuning_id);

/* Time every tuning-table entry on the given batched problem (forward and,
 * if grad_image != NULL, backward; inputs as for the batched calls, with the
 * workspace sized for the largest entry by inpc_batched_sizes) and record the
 * fastest for its shape bucket.  Synchronises ``stream``.  If cache_path is
 * not NULL the table of choices is merged into that JSON file.  Returns the
 * chosen tuning id (>= 0) or a negative error code; *best_ms receives its
 * time per call. */
int inpc_autotune(const float *xyz, const void *feat, int32_t feat_dtype, const float *opacity,
                  int64_t n_points, int32_t F, const inpc_view_t *views_host, int32_t n_views,
                  float t_threshold, float *image, float *t_final, void *saved,
                  size_t saved_bytes, const float *grad_image, float *grad_feat,
                  float *grad_opacity, void *ws, size_t ws_bytes, int32_t repeats,
                  const char *cache_path, float *best_ms, void *stream);

/* Load choices written by inpc_autotune from a JSON file (merged into the
 * in-process cache).  Returns the number of entries loaded or a negative code. */
int inpc_autotune_load(const char *cache_path);

/* Tuning id the library uses for this problem when settings.tuning_id == -1. */
int inpc_tuning_for(const inpc_view_t *views_host, int32_t n_views, int64_t n_points, int32_t F,
                    int32_t feat_dtype);

/* Tuning id of the last forward (plain or batched) that accepted ``saved``
 * (a device pointer, compared by address only and never dereferenced; the id
 * is recorded once the arguments pass validation, before the forward's work
 * is enqueued), or INPC_EINVAL if no forward of this process recorded one
 * (NULL, or the record was dropped after 4096 newer buffers).  Host only; no
 * device work. */
int inpc_saved_tuning(const void *saved);

/* ------------------------------------------------------ test/debug hooks */

/* Copy the sorted fragment list of a SAVE-mode forward to the host
 * (synchronises the stream).  saved and fwd_ws must be the buffers that
 * forward used, untouched since (fwd_ws may be NULL when keys_host is).  keys_host[i] = (global pixel << 32) | float32
 * bits of the view depth; ids_host[i] = 4*(view point) + corner, in sorted
 * order; *m_out = number of fragments (arrays of capacity cap; nothing is
 * copied if cap < *m_out).  n_blended_host (may be NULL) receives, per
 * packed pixel, how many splats the blend consumed.  Not for the hot path:
 * it allocates host staging memory. */
int inpc_debug_fragments(const inpc_view_t *views_host, int32_t n_views, int64_t n_points,
                         int32_t F, int32_t feat_dtype, const void *saved, size_t saved_bytes,
                         const void *fwd_ws, size_t fwd_ws_bytes, uint64_t *keys_host,
                         uint32_t *ids_host, int64_t cap, int64_t *m_out,
                         uint32_t *n_blended_host, void *stream);

/* Per-stage timing (measurement support, not part of the method).  Between
 * inpc_profile_begin() and inpc_profile_end() every stage of the calls above
 * records a pair of HIP events on its stream (so do not capture graphs while
 * profiling).  inpc_profile_end() waits for them and writes, per stage, the
 * summed milliseconds and the number of timed launches into arrays of
 * inpc_profile_stage_count() entries (either may be NULL).  Process-wide;
 * not meant for concurrent use from several host threads. */
int inpc_profile_stage_count(void);
const char *inpc_profile_stage_name(int32_t stage);
int inpc_profile_begin(void);
int inpc_profile_end(double *total_ms, int64_t *launches);

const char *inpc_error_string(int code);
const char *inpc_last_hip_error(void);
int inpc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* INPC_RASTER_H */
