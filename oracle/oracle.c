/*
 * Plain FP64 CPU oracle for INPC's differentiable bilinear point rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  The parity tests, the smoke check and the CPU
 * baseline of the benchmark call it; the product path never does.  It shares
 * no code, header, table or helper with the HIP library.
 *
 * It evaluates the plain per-pixel definition, slowly and in the paper's
 * order, with no blocking or fusion:
 *
 *   Projection (Section 3.4, Eq. 5): p = P V p_w for a pinhole camera.
 *   Bilinear splat (Section 3.4, Eq. 6): each point is splatted to the 2x2
 *     pixels whose centres are closest to (u, v), with opacity
 *     alpha = alpha_h (1-|u-u_i|)(1-|v-v_i|).
 *   Blending (Eq. 1, Section 2): per pixel, front to back in depth order,
 *     C = sum_i T_i alpha_i c_i with T_i = prod_{j<i}(1-alpha_j); accumulation
 *     stops once the remaining transmittance falls below tau (Appendix A.6).
 *   Backward (Appendix A.6): per-splat gradients of the blend, and per point a
 *     sum of its (at most four) splat gradients weighted by the bilinear
 *     weights, which is the chain rule through Eq. 6.
 *
 * Readings of the paper fixed here (the paper is silent on them):
 *   - pixel (x, y) has its centre at (x+0.5, y+0.5); the 2x2 block is anchored
 *     at x0 = floor(u-0.5), y0 = floor(v-0.5);
 *   - the depth d that orders splats is the view-space z, compared through its
 *     float32 bit pattern (identical to float order for z > 0);
 *   - a point is kept iff near < z < far and -1 < u < W+1, -1 < v < H+1;
 *   - corners outside the image or with a zero bilinear factor emit nothing,
 *     and the remaining weights are not renormalised;
 *   - equal depths inside a pixel are ordered by ascending splat id 4p+corner;
 *   - blending applies a splat, updates T, then stops if T < tau (strict);
 *     tau = 0 blends every splat;
 *   - the backward holds the forward's termination index fixed.
 *
 * Precision: the projection and the bilinear factors are float32 operations
 * in the exact order written below (no fused multiply-add: build with
 * -ffp-contract=off), because they decide which splats exist.  Everything
 * after that (weights, alpha, transmittance, colours, gradients) is float64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    float R[9];        /* world -> camera rotation, row-major */
    float t[3];        /* world -> camera translation */
    float fx, fy, cx, cy;
    int32_t width, height;
    float near_plane, far_plane;
} orc_camera_t;

static uint32_t f32_bits(float x) {
    uint32_t b;
    memcpy(&b, &x, sizeof b);
    return b;
}

static double feat_value(const void *feat, int bf16, int64_t row, int32_t F, int32_t f) {
    if (!bf16) return (double)((const float *)feat)[row * F + f];
    uint32_t b = (uint32_t)((const uint16_t *)feat)[row * F + f] << 16;
    float x;
    memcpy(&x, &b, sizeof x);
    return (double)x;
}

/*
 * Splats of one point (Eq. 5 and Eq. 6).  Writes up to four
 * (pixel index, depth bits, corner, weight) records; returns how many.
 */
static int splat_point(const float *pw, const orc_camera_t *c, int64_t *pix, uint32_t *zb,
                       int *corner, double *w) {
    float x = pw[0], y = pw[1], z = pw[2];
    float xc = ((c->R[0] * x + c->R[1] * y) + c->R[2] * z) + c->t[0];
    float yc = ((c->R[3] * x + c->R[4] * y) + c->R[5] * z) + c->t[1];
    float zc = ((c->R[6] * x + c->R[7] * y) + c->R[8] * z) + c->t[2];
    if (!(zc > c->near_plane && zc < c->far_plane)) return 0;
    float u = c->fx * (xc / zc) + c->cx;
    float v = c->fy * (yc / zc) + c->cy;
    if (!(u > -1.0f && u < (float)(c->width + 1))) return 0;
    if (!(v > -1.0f && v < (float)(c->height + 1))) return 0;
    float su = u - 0.5f, sv = v - 0.5f;
    int x0 = (int)floorf(su), y0 = (int)floorf(sv);
    float ax = su - (float)x0, ay = sv - (float)y0;
    float wx[2], wy[2];
    wx[0] = 1.0f - ax;
    wx[1] = ax;
    wy[0] = 1.0f - ay;
    wy[1] = ay;
    int k = 0;
    for (int cc = 0; cc < 4; ++cc) {
        int dx = cc & 1, dy = cc >> 1;
        int px = x0 + dx, py = y0 + dy;
        if (px < 0 || px >= c->width || py < 0 || py >= c->height) continue;
        if (!(wx[dx] > 0.0f) || !(wy[dy] > 0.0f)) continue;
        pix[k] = (int64_t)py * c->width + px;
        zb[k] = f32_bits(zc);
        corner[k] = cc;
        w[k] = (double)wx[dx] * (double)wy[dy];
        ++k;
    }
    return k;
}

/*
 * Emit every splat of points [0, n) in point order.  Writes at most ``cap``
 * records into pixel/zbits/id/weight (any may be NULL when cap == 0) and
 * returns the total number of splats.  id = 4*p + corner.
 */
int64_t orc_emit(const float *xyz, int64_t n, const orc_camera_t *cam, uint32_t *pixel,
                 uint32_t *zbits, uint32_t *id, double *weight, int64_t cap) {
    int64_t m = 0;
    for (int64_t p = 0; p < n; ++p) {
        int64_t pix[4];
        uint32_t zb[4];
        int corner[4];
        double w[4];
        int k = splat_point(xyz + 3 * p, cam, pix, zb, corner, w);
        for (int i = 0; i < k; ++i, ++m) {
            if (m >= cap) continue;
            pixel[m] = (uint32_t)pix[i];
            zbits[m] = zb[i];
            id[m] = (uint32_t)(4 * p + corner[i]);
            weight[m] = w[i];
        }
    }
    return m;
}

typedef struct {
    uint32_t zbits;
    uint32_t id;
    double w;
} orc_entry_t;

static int entry_cmp(const void *a, const void *b) {
    const orc_entry_t *x = (const orc_entry_t *)a, *y = (const orc_entry_t *)b;
    if (x->zbits != y->zbits) return x->zbits < y->zbits ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

/*
 * Per-pixel splat lists in depth order.  Input: the m splats from orc_emit.
 * Output: start[P+1] (list of pixel q is [start[q], start[q+1])) and the
 * concatenated lists, each sorted by (depth bits, id).  Returns 0, or -1 on
 * a pixel index outside [0, P) or an allocation failure.
 */
int orc_build_lists(int64_t P, int64_t m, const uint32_t *pixel, const uint32_t *zbits,
                    const uint32_t *id, const double *weight, int64_t *start, uint32_t *s_zbits,
                    uint32_t *s_id, double *s_w) {
    int64_t *fill = (int64_t *)calloc((size_t)P + 1, sizeof(int64_t));
    orc_entry_t *lists = (orc_entry_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(orc_entry_t));
    if (!fill || !lists) {
        free(fill);
        free(lists);
        return -1;
    }
    for (int64_t q = 0; q <= P; ++q) start[q] = 0;
    for (int64_t i = 0; i < m; ++i) {
        if ((int64_t)pixel[i] >= P) {
            free(fill);
            free(lists);
            return -1;
        }
        start[pixel[i] + 1] += 1;
    }
    for (int64_t q = 0; q < P; ++q) start[q + 1] += start[q];
    for (int64_t i = 0; i < m; ++i) {
        int64_t q = pixel[i];
        orc_entry_t e = {zbits[i], id[i], weight[i]};
        lists[start[q] + fill[q]++] = e;
    }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t q = 0; q < P; ++q) {
        int64_t len = start[q + 1] - start[q];
        if (len > 1) qsort(lists + start[q], (size_t)len, sizeof(orc_entry_t), entry_cmp);
    }
    for (int64_t i = 0; i < m; ++i) {
        s_zbits[i] = lists[i].zbits;
        s_id[i] = lists[i].id;
        s_w[i] = lists[i].w;
    }
    free(fill);
    free(lists);
    return 0;
}

/*
 * Forward blend of Eq. 1 per pixel over its sorted list.
 *   alpha_k = opa[p] * w_k, C += T alpha_k c_p, T *= (1 - alpha_k);
 *   stop after the splat that makes T < tau.
 * If n_override is given, pixel q blends exactly n_override[q] splats
 * instead (tau is then ignored for that pixel).  t_after (optional, [m])
 * receives the transmittance after every splat of every list, continuing
 * past the termination point, for the termination-ambiguity check.
 * Outputs: image [P,F], t_final [P], n_blended [P].
 */
void orc_blend_fwd(int64_t P, const int64_t *start, const uint32_t *s_id, const double *s_w,
                   const float *opa, const void *feat, int feat_bf16, int32_t F, double tau,
                   const int32_t *n_override, double *image, double *t_final, int32_t *n_blended,
                   double *t_after) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t q = 0; q < P; ++q) {
        double *C = image + q * F;
        for (int32_t f = 0; f < F; ++f) C[f] = 0.0;
        double T = 1.0, T_run = 1.0;
        int32_t n = 0;
        int done = 0;
        for (int64_t k = start[q]; k < start[q + 1]; ++k) {
            int64_t p = s_id[k] >> 2;
            double alpha = (double)opa[p] * s_w[k];
            if (n_override && n >= n_override[q]) done = 1;
            if (!done) {
                for (int32_t f = 0; f < F; ++f) C[f] += T * alpha * feat_value(feat, feat_bf16, p, F, f);
                T = T * (1.0 - alpha);
                n += 1;
                if (!n_override && T < tau) done = 1;
            }
            T_run = T_run * (1.0 - alpha);
            if (t_after) t_after[k] = T_run;
            if (done && !t_after) break;
        }
        t_final[q] = T;
        n_blended[q] = n;
    }
}

/*
 * Backward of orc_blend_fwd with the termination count n_blended held fixed.
 * For a pixel with blended splats 1..n, R_{n+1} = 0, Q_{n+1} = 1 and
 *   R_k = alpha_k c_k + (1 - alpha_k) R_{k+1},  Q_k = (1 - alpha_k) Q_{k+1},
 *   dL/dalpha_k = T_k sum_f g_f (c_{k,f} - R_{k+1,f}) - g_T T_k Q_{k+1},
 *   dL/dc_k     = T_k alpha_k g.
 * Per point (fixed corner order 0..3):
 *   grad_feat[p] = sum_c T_k alpha_k g_{pixel(k)},  grad_opa[p] = sum_c w_k dL/dalpha_k.
 * g_t may be NULL (treated as zero).  Returns 0, or -1 on allocation failure.
 */
int orc_blend_bwd(int64_t P, const int64_t *start, const uint32_t *s_id, const double *s_w,
                  const float *opa, const void *feat, int feat_bf16, int32_t F,
                  const int32_t *n_blended, const float *g_img, const float *g_t, int64_t N,
                  double *grad_feat, double *grad_opa) {
    size_t nf = (size_t)(4 * N > 0 ? 4 * N : 1);
    double *d_alpha = (double *)calloc(nf, sizeof(double));
    double *t_alpha = (double *)calloc(nf, sizeof(double));
    double *w_of = (double *)calloc(nf, sizeof(double));
    int64_t *pix_of = (int64_t *)malloc(nf * sizeof(int64_t));
    int rc = 0;
    if (!d_alpha || !t_alpha || !w_of || !pix_of) {
        rc = -1;
        goto out;
    }
    for (size_t i = 0; i < nf; ++i) pix_of[i] = -1;

#pragma omp parallel
    {
        double *R = (double *)malloc((size_t)(F > 0 ? F : 1) * sizeof(double));
        double *Tk = NULL;
        int64_t cap = 0;
#pragma omp for schedule(dynamic, 256)
        for (int64_t q = 0; q < P; ++q) {
            int64_t s = start[q];
            int32_t n = n_blended[q];
            for (int64_t k = s; k < start[q + 1]; ++k) {
                pix_of[s_id[k]] = q;
                w_of[s_id[k]] = s_w[k];
            }
            if (n == 0) continue;
            if (n > cap) {
                free(Tk);
                cap = n;
                Tk = (double *)malloc((size_t)cap * sizeof(double));
            }
            double T = 1.0;
            for (int32_t k = 0; k < n; ++k) {
                Tk[k] = T;
                double alpha = (double)opa[s_id[s + k] >> 2] * s_w[s + k];
                T = T * (1.0 - alpha);
            }
            for (int32_t f = 0; f < F; ++f) R[f] = 0.0;
            double Q = 1.0;
            double gT = g_t ? (double)g_t[q] : 0.0;
            const float *g = g_img + q * F;
            for (int32_t k = n - 1; k >= 0; --k) {
                uint32_t id = s_id[s + k];
                int64_t p = id >> 2;
                double alpha = (double)opa[p] * s_w[s + k];
                double acc = 0.0;
                for (int32_t f = 0; f < F; ++f)
                    acc += (double)g[f] * (feat_value(feat, feat_bf16, p, F, f) - R[f]);
                d_alpha[id] = Tk[k] * acc - gT * Tk[k] * Q;
                t_alpha[id] = Tk[k] * alpha;
                for (int32_t f = 0; f < F; ++f)
                    R[f] = alpha * feat_value(feat, feat_bf16, p, F, f) + (1.0 - alpha) * R[f];
                Q = (1.0 - alpha) * Q;
            }
        }
        free(R);
        free(Tk);
    }

#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
        double go = 0.0;
        for (int32_t f = 0; f < F; ++f) grad_feat[p * F + f] = 0.0;
        for (int c = 0; c < 4; ++c) {
            int64_t id = 4 * p + c;
            if (pix_of[id] < 0) continue;
            go += w_of[id] * d_alpha[id];
            const float *g = g_img + pix_of[id] * F;
            for (int32_t f = 0; f < F; ++f) grad_feat[p * F + f] += t_alpha[id] * (double)g[f];
        }
        grad_opa[p] = go;
    }
out:
    free(d_alpha);
    free(t_alpha);
    free(w_of);
    free(pix_of);
    return rc;
}

/*
 * Per-point blend weight for the probability-field updates (Section 3.1,
 * Eq. 2 and Eq. 3 use the transmitted blending weight b = alpha T of Eq. 1;
 * Appendix A.6 combines a point's per-splat weights in a sum weighted by the
 * bilinear weights).  With the termination count n_blended[q] of each pixel:
 *   b[p] = sum over the blended splats k of p of  w_k * T_k * alpha_k.
 * Points without blended splats get 0.
 */
void orc_blend_weight(int64_t P, const int64_t *start, const uint32_t *s_id, const double *s_w,
                      const float *opa, const int32_t *n_blended, int64_t N, double *bw) {
    for (int64_t p = 0; p < N; ++p) bw[p] = 0.0;
    /* serial over pixels: several pixels add into one point */
    for (int64_t q = 0; q < P; ++q) {
        double T = 1.0;
        for (int32_t k = 0; k < n_blended[q]; ++k) {
            int64_t i = start[q] + k;
            int64_t p = s_id[i] >> 2;
            double alpha = (double)opa[p] * s_w[i];
            bw[p] += s_w[i] * (T * alpha);
            T = T * (1.0 - alpha);
        }
    }
}

/* Number of OpenMP threads a parallel region of this library uses. */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the number of OpenMP threads of later parallel regions (n >= 1). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
