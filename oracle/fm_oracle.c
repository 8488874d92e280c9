/*
 * fm_oracle.c -- FP64 CPU oracle for the differentiable 2D Gaussian surfel
 * (2DGS) rasterizer: projection, ray-splat intersection, depth-ordered
 * front-to-back alpha compositing (the paper's Eq. 1, Sec. 3 "Preliminaries"),
 * with an analytic reverse-sweep backward, and the tile binning the GPU path
 * must reproduce bit for bit.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the HIP path.
 *
 * Everything is evaluated in FP64 from the FP32 inputs.  The rendering is a
 * per-pixel brute force: every non-culled surfel whose loose bounding box
 * contains the pixel is intersected exactly, candidates are taken in
 * (fp32(z), index) order, and compositing stops at the transmittance floor.
 * The loose box is only a candidate pre-filter; prefilter=0 disables it and
 * the result is identical (checked by the tests).
 *
 * Readings of the paper (it gives Eq. 1 only; the rest is the usual 2DGS
 * convention, restated here from its mathematics):
 *   - a surfel is a planar disk: centre mu, rotation q (w,x,y,z; normalised
 *     here), tangent scales (s_u, s_v), opacity sigma, RGB colour c;
 *   - the weight w_i(p) of Eq. 1 is evaluated by exact ray-splat intersection:
 *     the pixel ray meets the surfel plane at local coordinates (u, v), and
 *     G = exp(-(u^2+v^2)/2); alpha = min(alpha_max, sigma G); a candidate is
 *     skipped when u^2+v^2 > rho_max^2 or sigma G < alpha_min;
 *   - z_i of Eq. 1 is the camera-space depth of the surfel centre;
 *   - the normal output sums alpha T n_i with n_i the camera-space surfel
 *     normal turned to face the camera;
 *   - the image adds T_final * background; depth, normal, alpha do not.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double alpha_min, alpha_max, t_min, rho_max, near_z;
    double bg[3];
    double margin;    /* relative margin for r^2 and alpha threshold flags */
    double margin_t;  /* relative margin for the transmittance-floor flag */
    double cond_eps;  /* assumed relative perturbation of the constraint rows a, b */
    double cond_tol;  /* flag a pixel when the resulting alpha change may exceed this */
    int prefilter;    /* 1: loose-box candidate filter, 0: all surfels everywhere */
    int n_threads;    /* 0: OpenMP default */
} orc_params;

typedef struct {
    int valid;
    double qhat[4], qnorm;
    double Rs[9];            /* row-major rotation of the surfel frame */
    double p[3], tu[3], tv[3], n0[3];
    double sign;             /* +1 keeps n0, -1 flips it towards the camera */
    double H[9];             /* row-major 3x3, columns K s_u t_u, K s_v t_v, K p */
    double su, sv, sigma, col[3];
    double z;
    float kappa;
    int px0, px1, py0, py1;  /* exact pixel-centre bbox (R13), inclusive */
    int lx0, lx1, ly0, ly1;  /* loose candidate box, inclusive */
} surf_t;

static int fin(float v) { return isfinite(v); }

/*
 * Per-surfel projection.  The operation order is fixed (left-to-right sums,
 * no fused multiply-add) because the cull decisions, the depth key and the
 * pixel bbox must come out bit-identical on the GPU.  Compile with
 * -ffp-contract=off.
 */
static void preprocess(int i, int n, const float *mean, const float *quat, const float *scale,
                       const float *opacity, const float *color, int W, int Hh,
                       const float *intr, const float *vm, const orc_params *pp, surf_t *s)
{
    memset(s, 0, sizeof(*s));
    s->valid = 0;
    s->px0 = 1; s->px1 = 0; s->py0 = 1; s->py1 = 0;
    s->lx0 = 1; s->lx1 = 0; s->ly0 = 1; s->ly1 = 0;
    float raw[13] = {mean[i], mean[n + i], mean[2 * n + i], quat[i], quat[n + i], quat[2 * n + i],
                     quat[3 * n + i], scale[i], scale[n + i], opacity[i], color[i], color[n + i],
                     color[2 * n + i]};
    for (int k = 0; k < 13; ++k)
        if (!fin(raw[k])) return;
    double mx = mean[i], my = mean[n + i], mz = mean[2 * n + i];
    double qw = quat[i], qx = quat[n + i], qy = quat[2 * n + i], qz = quat[3 * n + i];
    double su = scale[i], sv = scale[n + i];
    double sigma = opacity[i];
    if (!(su > 0.0) || !(sv > 0.0)) return;
    double qn = qw * qw + qx * qx + qy * qy + qz * qz;
    if (!(qn > 0.0)) return;
    double qnorm = sqrt(qn);
    double w = qw / qnorm, x = qx / qnorm, y = qy / qnorm, z = qz / qnorm;
    double Rs[9];
    Rs[0] = 1.0 - 2.0 * (y * y + z * z);
    Rs[1] = 2.0 * (x * y - w * z);
    Rs[2] = 2.0 * (x * z + w * y);
    Rs[3] = 2.0 * (x * y + w * z);
    Rs[4] = 1.0 - 2.0 * (x * x + z * z);
    Rs[5] = 2.0 * (y * z - w * x);
    Rs[6] = 2.0 * (x * z - w * y);
    Rs[7] = 2.0 * (y * z + w * x);
    Rs[8] = 1.0 - 2.0 * (x * x + y * y);
    double R[9] = {vm[0], vm[1], vm[2], vm[4], vm[5], vm[6], vm[8], vm[9], vm[10]};
    double t[3] = {vm[3], vm[7], vm[11]};
    double p[3], tu[3], tv[3], n0[3];
    for (int r = 0; r < 3; ++r) {
        p[r] = R[3 * r] * mx + R[3 * r + 1] * my + R[3 * r + 2] * mz + t[r];
        tu[r] = R[3 * r] * Rs[0] + R[3 * r + 1] * Rs[3] + R[3 * r + 2] * Rs[6];
        tv[r] = R[3 * r] * Rs[1] + R[3 * r + 1] * Rs[4] + R[3 * r + 2] * Rs[7];
        n0[r] = R[3 * r] * Rs[2] + R[3 * r + 1] * Rs[5] + R[3 * r + 2] * Rs[8];
    }
    double depth = p[2];
    if (!(depth > pp->near_z)) return;
    if (!(sigma > pp->alpha_min)) return;
    double fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
    double M[9];
    for (int r = 0; r < 3; ++r) {
        M[3 * r + 0] = su * tu[r];
        M[3 * r + 1] = sv * tv[r];
        M[3 * r + 2] = p[r];
    }
    double H[9];
    for (int c = 0; c < 3; ++c) {
        H[c] = fx * M[c] + cx * M[6 + c];
        H[3 + c] = fy * M[3 + c] + cy * M[6 + c];
        H[6 + c] = M[6 + c];
    }
    double rho2 = pp->rho_max * pp->rho_max;
    /* dual conic of the support ellipse: rho^2 (h_u h_u^T + h_v h_v^T) - h_c h_c^T */
    double C00 = rho2 * (H[0] * H[0] + H[1] * H[1]) - H[2] * H[2];
    double C02 = rho2 * (H[0] * H[6] + H[1] * H[7]) - H[2] * H[8];
    double C11 = rho2 * (H[3] * H[3] + H[4] * H[4]) - H[5] * H[5];
    double C12 = rho2 * (H[3] * H[6] + H[4] * H[7]) - H[5] * H[8];
    double C22 = rho2 * (H[6] * H[6] + H[7] * H[7]) - H[8] * H[8];
    if (!(C22 < 0.0)) return;  /* support disk not entirely in front of the camera */
    double dx = C02 * C02 - C00 * C22;
    double dy = C12 * C12 - C11 * C22;
    if (!(dx >= 0.0) || !(dy >= 0.0)) return;
    double sx = sqrt(dx), sy = sqrt(dy);
    double xa = (C02 - sx) / C22, xb = (C02 + sx) / C22;
    double ya = (C12 - sy) / C22, yb = (C12 + sy) / C22;
    double xlo = xa < xb ? xa : xb, xhi = xa < xb ? xb : xa;
    double ylo = ya < yb ? ya : yb, yhi = ya < yb ? yb : ya;
    double c0 = ceil(xlo - 0.5), c1 = floor(xhi - 0.5);
    double r0 = ceil(ylo - 0.5), r1 = floor(yhi - 0.5);
    if (c0 < 0.0) c0 = 0.0;
    if (r0 < 0.0) r0 = 0.0;
    if (c1 > (double)(W - 1)) c1 = (double)(W - 1);
    if (r1 > (double)(Hh - 1)) r1 = (double)(Hh - 1);
    double dotnp = n0[0] * p[0] + n0[1] * p[1] + n0[2] * p[2];

    s->valid = 1;
    memcpy(s->Rs, Rs, sizeof(Rs));
    s->qhat[0] = w; s->qhat[1] = x; s->qhat[2] = y; s->qhat[3] = z;
    s->qnorm = qnorm;
    memcpy(s->p, p, sizeof(p));
    memcpy(s->tu, tu, sizeof(tu));
    memcpy(s->tv, tv, sizeof(tv));
    memcpy(s->n0, n0, sizeof(n0));
    s->sign = dotnp < 0.0 ? 1.0 : -1.0;
    memcpy(s->H, H, sizeof(H));
    s->su = su; s->sv = sv; s->sigma = sigma;
    s->col[0] = color[i]; s->col[1] = color[n + i]; s->col[2] = color[2 * n + i];
    s->z = depth;
    s->kappa = (float)depth;
    if (c0 <= c1 && r0 <= r1) {
        s->px0 = (int)c0; s->px1 = (int)c1; s->py0 = (int)r0; s->py1 = (int)r1;
    }
    /* loose candidate box: the disk lies in the ball of radius rho_max*max(s)
     * around p; project the axis-aligned cube around that ball. */
    double rad = pp->rho_max * (su > sv ? su : sv);
    if (p[2] - rad <= 0.0) {
        s->lx0 = 0; s->lx1 = W - 1; s->ly0 = 0; s->ly1 = Hh - 1;
    } else {
        double zc[2] = {p[2] - rad, p[2] + rad};
        double xs[2] = {p[0] - rad, p[0] + rad};
        double ys[2] = {p[1] - rad, p[1] + rad};
        double ux = -INFINITY, lx = INFINITY, uy = -INFINITY, ly = INFINITY;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                double vx = fx * xs[a] / zc[b] + cx, vy = fy * ys[a] / zc[b] + cy;
                if (vx < lx) lx = vx;
                if (vx > ux) ux = vx;
                if (vy < ly) ly = vy;
                if (vy > uy) uy = vy;
            }
        double a0 = floor(lx - 0.5) - 1.0, a1 = ceil(ux - 0.5) + 1.0;
        double b0 = floor(ly - 0.5) - 1.0, b1 = ceil(uy - 0.5) + 1.0;
        if (a0 < 0.0) a0 = 0.0;
        if (b0 < 0.0) b0 = 0.0;
        if (a1 > W - 1) a1 = W - 1;
        if (b1 > Hh - 1) b1 = Hh - 1;
        if (a0 <= a1 && b0 <= b1) {
            s->lx0 = (int)a0; s->lx1 = (int)a1; s->ly0 = (int)b0; s->ly1 = (int)b1;
        }
    }
    if (!pp->prefilter) {
        s->lx0 = 0; s->lx1 = W - 1; s->ly0 = 0; s->ly1 = Hh - 1;
    }
}

/* candidate order: ascending fp32 depth key, ties by surfel index */
static const surf_t *g_sort_base;
static int cmp_order(const void *a, const void *b)
{
    int ia = *(const int *)a, ib = *(const int *)b;
    float ka = g_sort_base[ia].kappa, kb = g_sort_base[ib].kappa;
    if (ka < kb) return -1;
    if (ka > kb) return 1;
    return (ia > ib) - (ia < ib);
}

/* Intersection of the ray through pixel centre (x, y) with the surfel plane.
 * Returns 0 if the ray is parallel to the plane. */
static int intersect(const surf_t *s, double x, double y, double *a, double *b, double *w,
                     double *u, double *v, double *r2)
{
    const double *H = s->H;
    for (int j = 0; j < 3; ++j) {
        a[j] = H[j] - x * H[6 + j];
        b[j] = H[3 + j] - y * H[6 + j];
    }
    w[0] = a[1] * b[2] - a[2] * b[1];
    w[1] = a[2] * b[0] - a[0] * b[2];
    w[2] = a[0] * b[1] - a[1] * b[0];
    if (w[2] == 0.0) return 0;
    *u = w[0] / w[2];
    *v = w[1] / w[2];
    *r2 = (*u) * (*u) + (*v) * (*v);
    return 1;
}

typedef struct {
    int n;               /* surfels */
    surf_t *s;
    int *order;          /* visible surfels sorted by (kappa, i) */
    int n_vis;
    int bw, bh, nbx, nby;/* candidate blocks */
    int **blk;           /* per block: indices into order (sorted) */
    int *blk_n;
} scene_t;

#define BLK 16

static int build_scene(scene_t *sc, int n, const float *mean, const float *quat, const float *scale,
                       const float *opacity, const float *color, int W, int H, const float *intr,
                       const float *vm, const orc_params *pp)
{
    memset(sc, 0, sizeof(*sc));
    sc->n = n;
    sc->s = (surf_t *)malloc(sizeof(surf_t) * (size_t)(n > 0 ? n : 1));
    sc->order = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!sc->s || !sc->order) return -1;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        preprocess(i, n, mean, quat, scale, opacity, color, W, H, intr, vm, pp, &sc->s[i]);
    int m = 0;
    for (int i = 0; i < n; ++i)
        if (sc->s[i].valid) sc->order[m++] = i;
    sc->n_vis = m;
    g_sort_base = sc->s;
    qsort(sc->order, (size_t)m, sizeof(int), cmp_order);
    sc->bw = BLK; sc->bh = BLK;
    sc->nbx = (W + BLK - 1) / BLK;
    sc->nby = (H + BLK - 1) / BLK;
    int nb = sc->nbx * sc->nby;
    sc->blk = (int **)calloc((size_t)(nb > 0 ? nb : 1), sizeof(int *));
    sc->blk_n = (int *)calloc((size_t)(nb > 0 ? nb : 1), sizeof(int));
    if (!sc->blk || !sc->blk_n) return -1;
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nb; ++b) {
        int bx = b % sc->nbx, by = b / sc->nbx;
        int x0 = bx * BLK, x1 = x0 + BLK - 1, y0 = by * BLK, y1 = y0 + BLK - 1;
        int cnt = 0;
        for (int k = 0; k < m; ++k) {
            const surf_t *s = &sc->s[sc->order[k]];
            if (s->lx0 <= x1 && s->lx1 >= x0 && s->ly0 <= y1 && s->ly1 >= y0) ++cnt;
        }
        int *lst = (int *)malloc(sizeof(int) * (size_t)(cnt > 0 ? cnt : 1));
        if (!lst) { fail = 1; continue; }
        cnt = 0;
        for (int k = 0; k < m; ++k) {
            const surf_t *s = &sc->s[sc->order[k]];
            if (s->lx0 <= x1 && s->lx1 >= x0 && s->ly0 <= y1 && s->ly1 >= y0) lst[cnt++] = sc->order[k];
        }
        sc->blk[b] = lst;
        sc->blk_n[b] = cnt;
    }
    return fail ? -1 : 0;
}

static void free_scene(scene_t *sc)
{
    int nb = sc->nbx * sc->nby;
    if (sc->blk)
        for (int b = 0; b < nb; ++b) free(sc->blk[b]);
    free(sc->blk);
    free(sc->blk_n);
    free(sc->s);
    free(sc->order);
}

static int near_rel(double v, double thr, double m) { return fabs(v - thr) <= m * fabs(thr); }

typedef struct {
    int idx;
    double alpha, at, G, T;
    double a[3], b[3], w[3], u, v;
    int clamped;
} contrib_t;

/*
 * Composite one pixel.  Fills up to cap contributors (front to back) into
 * list (if non-NULL); returns the number of contributors, sets *T_out and the
 * flag for threshold proximity.
 */
static int composite_pixel(const scene_t *sc, const orc_params *pp, int col, int row, int W,
                           double out[8], double *T_out, int *flag, contrib_t *list, int cap,
                           int64_t *n_eval)
{
    int b = (row / BLK) * sc->nbx + (col / BLK);
    const int *lst = sc->blk[b];
    int ln = sc->blk_n[b];
    double x = col + 0.5, y = row + 0.5;
    double rho2 = pp->rho_max * pp->rho_max;
    double T = 1.0;
    int m = 0;
    int fl = 0;
    for (int k = 0; k < 8; ++k) out[k] = 0.0;
    int64_t ne = 0;
    (void)W;
    for (int k = 0; k < ln; ++k) {
        const surf_t *s = &sc->s[lst[k]];
        if (col < s->lx0 || col > s->lx1 || row < s->ly0 || row > s->ly1) continue;
        double a[3], bb[3], w[3], u, v, r2;
        if (!intersect(s, x, y, a, bb, w, &u, &v, &r2)) {
            /* ray parallel to the surfel plane: no intersection; fully degenerate
             * constraint rows are flagged */
            if (w[0] == 0.0 && w[1] == 0.0) fl = 1;
            continue;
        }
        if (near_rel(r2, rho2, pp->margin)) fl = 1;
        if (r2 > rho2) continue;
        double G = exp(-0.5 * r2);
        double at = s->sigma * G;
        if (near_rel(at, pp->alpha_min, pp->margin)) fl = 1;
        if (at < pp->alpha_min) continue;
        if (near_rel(at, pp->alpha_max, pp->margin)) fl = 1;
        if (pp->cond_eps > 0.0) {
            /* conditioning of alpha w.r.t. relative perturbations of the two
             * plane-ray constraint rows a, b: near-grazing rays make u, v (and
             * so alpha) arbitrarily sensitive to rounding */
            double gw[3] = {2.0 * u / w[2], 2.0 * v / w[2], -2.0 * r2 / w[2]};
            double da[3] = {bb[1] * gw[2] - bb[2] * gw[1], bb[2] * gw[0] - bb[0] * gw[2],
                            bb[0] * gw[1] - bb[1] * gw[0]};
            double db[3] = {gw[1] * a[2] - gw[2] * a[1], gw[2] * a[0] - gw[0] * a[2],
                            gw[0] * a[1] - gw[1] * a[0]};
            double S = 0.0;
            for (int j = 0; j < 3; ++j) S += fabs(da[j] * a[j]) + fabs(db[j] * bb[j]);
            double zs = s->z > 1.0 ? s->z : 1.0;
            if (0.5 * at * S * pp->cond_eps * zs > pp->cond_tol) fl = 1;
        }
        int clamped = at > pp->alpha_max;
        double alpha = clamped ? pp->alpha_max : at;
        double tn = T * (1.0 - alpha);
        ++ne;
        if (near_rel(tn, pp->t_min, pp->margin_t)) fl = 1;
        if (tn < pp->t_min) break;
        double wgt = alpha * T;
        out[0] += s->col[0] * wgt;
        out[1] += s->col[1] * wgt;
        out[2] += s->col[2] * wgt;
        out[3] += s->z * wgt;
        out[4] += s->sign * s->n0[0] * wgt;
        out[5] += s->sign * s->n0[1] * wgt;
        out[6] += s->sign * s->n0[2] * wgt;
        out[7] += wgt;
        if (list) {
            if (m < cap) {
                contrib_t *c = &list[m];
                c->idx = lst[k];
                c->alpha = alpha; c->at = at; c->G = G; c->T = T;
                memcpy(c->a, a, sizeof(a)); memcpy(c->b, bb, sizeof(bb)); memcpy(c->w, w, sizeof(w));
                c->u = u; c->v = v;
                c->clamped = clamped;
            }
        }
        ++m;
        T = tn;
    }
    *T_out = T;
    *flag = fl;
    if (n_eval) *n_eval = ne;
    return m;
}

/*
 * Forward render of one view.  Outputs are planar (channel-major) over the
 * W*H pixels: rgb[3][WH], depth[WH], normal[3][WH], alpha[WH], t_final[WH],
 * n_contrib[WH] (number of composited surfels), flags[WH] (1 when some
 * decision at that pixel lies within the margin of its threshold).
 * n_useful receives the total number of composited (pixel, surfel) pairs.
 */
int orc_render(int n, const float *mean, const float *quat, const float *scale, const float *opacity,
               const float *color, int W, int H, const float *intr, const float *viewmat,
               const orc_params *pp, double *rgb, double *depth, double *normal, double *alpha,
               double *t_final, int32_t *n_contrib, uint8_t *flags, int64_t *n_useful)
{
#ifdef _OPENMP
    if (pp->n_threads > 0) omp_set_num_threads(pp->n_threads);
#endif
    scene_t sc;
    if (build_scene(&sc, n, mean, quat, scale, opacity, color, W, H, intr, viewmat, pp)) {
        free_scene(&sc);
        return -1;
    }
    int64_t total = 0;
    const size_t np = (size_t)W * H;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : total)
    for (int row = 0; row < H; ++row) {
        for (int col = 0; col < W; ++col) {
            double o[8], T;
            int fl;
            int m = composite_pixel(&sc, pp, col, row, W, o, &T, &fl, NULL, 0, NULL);
            size_t q = (size_t)row * W + col;
            rgb[q] = o[0] + T * pp->bg[0];
            rgb[np + q] = o[1] + T * pp->bg[1];
            rgb[2 * np + q] = o[2] + T * pp->bg[2];
            depth[q] = o[3];
            normal[q] = o[4];
            normal[np + q] = o[5];
            normal[2 * np + q] = o[6];
            alpha[q] = o[7];
            if (t_final) t_final[q] = T;
            if (n_contrib) n_contrib[q] = m;
            if (flags) flags[q] = (uint8_t)fl;
            total += m;
        }
    }
    if (n_useful) *n_useful = total;
    free_scene(&sc);
    return 0;
}

/*
 * Pruning scores of one view for map fusion (Sec. 3.3, "Map Fusion": the map
 * is rendered from the keyframe and primitives that contribute to pixels
 * with a high reconstruction error are removed).  For every pixel with
 * mask[q] != 0, each surfel composited there adds its weight alpha T (its
 * contribution in Eq. 1) to score[idx]; score[n] is ADDED into.
 */
int orc_contrib_scores(int n, const float *mean, const float *quat, const float *scale, const float *opacity,
                       const float *color, int W, int H, const float *intr, const float *viewmat,
                       const orc_params *pp, const uint8_t *mask, double *score)
{
#ifdef _OPENMP
    if (pp->n_threads > 0) omp_set_num_threads(pp->n_threads);
    int nt = omp_get_max_threads();
#else
    int nt = 1;
#endif
    scene_t sc;
    if (build_scene(&sc, n, mean, quat, scale, opacity, color, W, H, intr, viewmat, pp)) {
        free_scene(&sc);
        return -1;
    }
    double *acc = (double *)calloc((size_t)nt * (size_t)(n > 0 ? n : 1), sizeof(double));
    if (!acc) { free_scene(&sc); return -1; }
    int fail = 0;
#pragma omp parallel
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *my = acc + (size_t)tid * n;
        int cap = 1024;
        contrib_t *list = (contrib_t *)malloc(sizeof(contrib_t) * cap);
#pragma omp for schedule(dynamic, 4)
        for (int row = 0; row < H; ++row) {
            for (int col = 0; col < W; ++col) {
                if (!mask[(size_t)row * W + col]) continue;
                double o[8], T;
                int fl, m;
                for (;;) {
                    m = composite_pixel(&sc, pp, col, row, W, o, &T, &fl, list, cap, NULL);
                    if (m <= cap || !list) break;
                    cap = m * 2;
                    free(list);
                    list = (contrib_t *)malloc(sizeof(contrib_t) * cap);
                }
                if (!list) { fail = 1; continue; }
                for (int k = 0; k < m; ++k) my[list[k].idx] += list[k].alpha * list[k].T;
            }
        }
        free(list);
    }
    for (int t = 0; t < nt; ++t)
        for (int i = 0; i < n; ++i) score[i] += acc[(size_t)t * n + i];
    free(acc);
    free_scene(&sc);
    return fail ? -1 : 0;
}

/* dL/d(unit quaternion) from dL/dR for the rotation matrix written above */
static void drot_dq(const double q[4], const double G[9], double dq[4])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    dq[0] = 2.0 * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
    dq[1] = 2.0 * (y * G[1] + z * G[2] + y * G[3] - 2.0 * x * G[4] - w * G[5] + z * G[6] + w * G[7] -
                   2.0 * x * G[8]);
    dq[2] = 2.0 * (-2.0 * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] -
                   2.0 * y * G[8]);
    dq[3] = 2.0 * (-2.0 * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.0 * z * G[4] + y * G[5] +
                   x * G[6] + y * G[7]);
}

#define NG 17 /* per-surfel screen-space gradient: dH[9], dsigma, dc[3], dn[3], dz */

/*
 * Backward of one view.  g_* are dL/d(outputs) in the forward's planar
 * layout (rgb includes the background term).  Gradients are ADDED into the
 * double arrays d_mean[3][n], d_quat[4][n], d_scale[2][n], d_opacity[n],
 * d_color[3][n] and d_viewmat[12] (dL/d[R|t], row-major).  Culled surfels,
 * the rho cut, the alpha_min skip, the alpha_max clamp and the
 * transmittance stop carry no gradient.
 */
int orc_render_backward(int n, const float *mean, const float *quat, const float *scale,
                        const float *opacity, const float *color, int W, int H, const float *intr,
                        const float *viewmat, const orc_params *pp, const double *g_rgb,
                        const double *g_depth, const double *g_normal, const double *g_alpha,
                        double *d_mean, double *d_quat, double *d_scale, double *d_opacity,
                        double *d_color, double *d_viewmat)
{
#ifdef _OPENMP
    if (pp->n_threads > 0) omp_set_num_threads(pp->n_threads);
    int nt = omp_get_max_threads();
#else
    int nt = 1;
#endif
    scene_t sc;
    if (build_scene(&sc, n, mean, quat, scale, opacity, color, W, H, intr, viewmat, pp)) {
        free_scene(&sc);
        return -1;
    }
    double *acc = (double *)calloc((size_t)nt * (size_t)(n > 0 ? n : 1) * NG, sizeof(double));
    if (!acc) { free_scene(&sc); return -1; }
    const size_t np = (size_t)W * H;
    int fail = 0;
#pragma omp parallel
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        double *my = acc + (size_t)tid * n * NG;
        int cap = 1024;
        contrib_t *list = (contrib_t *)malloc(sizeof(contrib_t) * cap);
#pragma omp for schedule(dynamic, 4)
        for (int row = 0; row < H; ++row) {
            for (int col = 0; col < W; ++col) {
                size_t q = (size_t)row * W + col;
                double gC[3] = {g_rgb[q], g_rgb[np + q], g_rgb[2 * np + q]};
                double gD = g_depth[q];
                double gN[3] = {g_normal[q], g_normal[np + q], g_normal[2 * np + q]};
                double gA = g_alpha[q];
                if (gC[0] == 0.0 && gC[1] == 0.0 && gC[2] == 0.0 && gD == 0.0 && gN[0] == 0.0 &&
                    gN[1] == 0.0 && gN[2] == 0.0 && gA == 0.0)
                    continue;
                double o[8], T;
                int fl;
                int m;
                for (;;) {
                    m = composite_pixel(&sc, pp, col, row, W, o, &T, &fl, list, cap, NULL);
                    if (m <= cap || !list) break;
                    cap = m * 2;
                    free(list);
                    list = (contrib_t *)malloc(sizeof(contrib_t) * cap);
                }
                if (!list) { fail = 1; continue; }
                double x = col + 0.5, y = row + 0.5;
                /* reverse sweep: V = value of the suffix behind the current surfel,
                 * per unit transmittance; starts at the background term */
                double V = gC[0] * pp->bg[0] + gC[1] * pp->bg[1] + gC[2] * pp->bg[2];
                for (int k = m - 1; k >= 0; --k) {
                    const contrib_t *c = &list[k];
                    const surf_t *s = &sc.s[c->idx];
                    double nk[3] = {s->sign * s->n0[0], s->sign * s->n0[1], s->sign * s->n0[2]};
                    double f = gC[0] * s->col[0] + gC[1] * s->col[1] + gC[2] * s->col[2] + gD * s->z +
                               gN[0] * nk[0] + gN[1] * nk[1] + gN[2] * nk[2] + gA;
                    double dalpha = c->T * (f - V);
                    double wgt = c->alpha * c->T;
                    double *g = my + (size_t)c->idx * NG;
                    g[10] += gC[0] * wgt;
                    g[11] += gC[1] * wgt;
                    g[12] += gC[2] * wgt;
                    g[13] += gN[0] * wgt;
                    g[14] += gN[1] * wgt;
                    g[15] += gN[2] * wgt;
                    g[16] += gD * wgt;
                    V = f * c->alpha + (1.0 - c->alpha) * V;
                    if (c->clamped) continue;
                    g[9] += dalpha * c->G;
                    double dG = dalpha * s->sigma;
                    double dr2 = -0.5 * c->G * dG;
                    double du = 2.0 * c->u * dr2, dv = 2.0 * c->v * dr2;
                    double w2 = c->w[2];
                    double gw[3] = {du / w2, dv / w2, -(du * c->u + dv * c->v) / w2};
                    /* w = a x b: dL/da = b x gw, dL/db = gw x a */
                    double da[3] = {c->b[1] * gw[2] - c->b[2] * gw[1], c->b[2] * gw[0] - c->b[0] * gw[2],
                                    c->b[0] * gw[1] - c->b[1] * gw[0]};
                    double db[3] = {gw[1] * c->a[2] - gw[2] * c->a[1], gw[2] * c->a[0] - gw[0] * c->a[2],
                                    gw[0] * c->a[1] - gw[1] * c->a[0]};
                    for (int j = 0; j < 3; ++j) {
                        g[j] += da[j];
                        g[3 + j] += db[j];
                        g[6 + j] += -x * da[j] - y * db[j];
                    }
                }
            }
        }
        free(list);
    }
    /* reduce per-thread screen-space gradients and apply the projection chain rule */
    double fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
    double R[9] = {viewmat[0], viewmat[1], viewmat[2], viewmat[4], viewmat[5], viewmat[6],
                   viewmat[8], viewmat[9], viewmat[10]};
    double dV[12] = {0};
    for (int i = 0; i < n; ++i) {
        const surf_t *s = &sc.s[i];
        if (!s->valid) continue;
        double g[NG] = {0};
        for (int t = 0; t < nt; ++t)
            for (int k = 0; k < NG; ++k) g[k] += acc[((size_t)t * n + i) * NG + k];
        /* H = K M, M = [s_u t_u | s_v t_v | p]  ->  dM = K^T dH */
        double dM[9];
        for (int c = 0; c < 3; ++c) {
            dM[c] = fx * g[c];
            dM[3 + c] = fy * g[3 + c];
            dM[6 + c] = cx * g[c] + cy * g[3 + c] + g[6 + c];
        }
        double dp[3] = {dM[2], dM[5], dM[8] + g[16]};
        double dtu[3] = {s->su * dM[0], s->su * dM[3], s->su * dM[6]};
        double dtv[3] = {s->sv * dM[1], s->sv * dM[4], s->sv * dM[7]};
        double dsu = s->tu[0] * dM[0] + s->tu[1] * dM[3] + s->tu[2] * dM[6];
        double dsv = s->tv[0] * dM[1] + s->tv[1] * dM[4] + s->tv[2] * dM[7];
        double dn0[3] = {s->sign * g[13], s->sign * g[14], s->sign * g[15]};
        /* p = R mu + t ; t_u,t_v,n0 = R * columns of R_s */
        double mu[3] = {mean[i], mean[n + i], mean[2 * n + i]};
        double dRs[9] = {0};
        for (int c = 0; c < 3; ++c) {
            d_mean[c * n + i] += R[c] * dp[0] + R[3 + c] * dp[1] + R[6 + c] * dp[2];
            double rt_u = R[c] * dtu[0] + R[3 + c] * dtu[1] + R[6 + c] * dtu[2];
            double rt_v = R[c] * dtv[0] + R[3 + c] * dtv[1] + R[6 + c] * dtv[2];
            double rt_n = R[c] * dn0[0] + R[3 + c] * dn0[1] + R[6 + c] * dn0[2];
            dRs[3 * c + 0] = rt_u;
            dRs[3 * c + 1] = rt_v;
            dRs[3 * c + 2] = rt_n;
        }
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c)
                dV[4 * r + c] += dp[r] * mu[c] + dtu[r] * s->Rs[3 * c] + dtv[r] * s->Rs[3 * c + 1] +
                                 dn0[r] * s->Rs[3 * c + 2];
            dV[4 * r + 3] += dp[r];
        }
        double dqh[4];
        drot_dq(s->qhat, dRs, dqh);
        double dot = dqh[0] * s->qhat[0] + dqh[1] * s->qhat[1] + dqh[2] * s->qhat[2] + dqh[3] * s->qhat[3];
        for (int k = 0; k < 4; ++k) d_quat[k * n + i] += (dqh[k] - s->qhat[k] * dot) / s->qnorm;
        d_scale[i] += dsu;
        d_scale[n + i] += dsv;
        d_opacity[i] += g[9];
        d_color[i] += g[10];
        d_color[n + i] += g[11];
        d_color[2 * n + i] += g[12];
    }
    for (int k = 0; k < 12; ++k) d_viewmat[k] += dV[k];
    free(acc);
    free_scene(&sc);
    return fail ? -1 : 0;
}

/*
 * Whether a surfel reaches a pixel of tile (a, b): some pixel centre of the
 * tile inside the image where the ray meets the surfel plane inside the
 * support (r^2 <= rho_max^2) with sigma G >= alpha_min -- the two per-pixel
 * tests of the compositing, before any transmittance stop.  A pair of the
 * bbox list whose tile no pixel passes cannot contribute to any pixel.
 */
static int tile_reached(const surf_t *s, const orc_params *pp, int a, int b, int tile_w, int tile_h, int W,
                        int H)
{
    double rho2 = pp->rho_max * pp->rho_max;
    for (int row = b * tile_h; row < (b + 1) * tile_h && row < H; ++row)
        for (int col = a * tile_w; col < (a + 1) * tile_w && col < W; ++col) {
            double aa[3], bb[3], w[3], u, v, r2;
            if (!intersect(s, col + 0.5, row + 0.5, aa, bb, w, &u, &v, &r2)) continue;
            if (r2 > rho2) continue;
            if (s->sigma * exp(-0.5 * r2) < pp->alpha_min) continue;
            return 1;
        }
    return 0;
}

/*
 * Tile binning of one view.  For every surfel surviving the culls, the tiles
 * covered by its pixel-centre bbox are listed; pairs are ordered by
 * (tile, fp32 depth key, surfel index).  Outputs:
 *   rect[4n]      tx0, ty0, tx1, ty1 per surfel (-1 when it covers no tile),
 *   kappa[n]      bits of the fp32 depth key (0 for culled surfels),
 *   pair_tile / pair_surf (capacity cap), *n_pairs,
 *   tile_start / tile_end [tiles_x * tiles_y] half-open ranges,
 *   pair_reached  (may be NULL) 1 when the pair's surfel reaches a pixel of
 *                 the pair's tile (tile_reached), else 0.
 */
typedef struct { uint32_t tile; float kappa; int32_t idx; } pair_t;
static int cmp_pair(const void *a, const void *b)
{
    const pair_t *p = (const pair_t *)a, *q = (const pair_t *)b;
    if (p->tile != q->tile) return p->tile < q->tile ? -1 : 1;
    if (p->kappa != q->kappa) return p->kappa < q->kappa ? -1 : 1;
    return (p->idx > q->idx) - (p->idx < q->idx);
}

int orc_bin(int n, const float *mean, const float *quat, const float *scale, const float *opacity,
            const float *color, int W, int H, const float *intr, const float *viewmat,
            const orc_params *pp, int tile_w, int tile_h, int32_t *rect, uint32_t *kappa,
            int64_t *n_pairs, uint32_t *pair_tile, uint32_t *pair_surf, int64_t cap,
            uint32_t *tile_start, uint32_t *tile_end, uint8_t *pair_reached)
{
    int tx = (W + tile_w - 1) / tile_w, ty = (H + tile_h - 1) / tile_h;
    surf_t *s = (surf_t *)malloc(sizeof(surf_t) * (size_t)(n > 0 ? n : 1));
    if (!s) return -1;
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        preprocess(i, n, mean, quat, scale, opacity, color, W, H, intr, viewmat, pp, &s[i]);
        if (s[i].valid && s[i].px0 <= s[i].px1 && s[i].py0 <= s[i].py1) {
            int a0 = s[i].px0 / tile_w, a1 = s[i].px1 / tile_w;
            int b0 = s[i].py0 / tile_h, b1 = s[i].py1 / tile_h;
            rect[4 * i] = a0; rect[4 * i + 1] = b0; rect[4 * i + 2] = a1; rect[4 * i + 3] = b1;
            total += (int64_t)(a1 - a0 + 1) * (b1 - b0 + 1);
        } else {
            rect[4 * i] = rect[4 * i + 1] = rect[4 * i + 2] = rect[4 * i + 3] = -1;
        }
        uint32_t bits = 0;
        if (s[i].valid) memcpy(&bits, &s[i].kappa, 4);
        kappa[i] = bits;
    }
    *n_pairs = total;
    if (total > cap) { free(s); return 2; }
    pair_t *pr = (pair_t *)malloc(sizeof(pair_t) * (size_t)(total > 0 ? total : 1));
    if (!pr) { free(s); return -1; }
    int64_t k = 0;
    for (int i = 0; i < n; ++i) {
        if (rect[4 * i] < 0) continue;
        for (int b = rect[4 * i + 1]; b <= rect[4 * i + 3]; ++b)
            for (int a = rect[4 * i]; a <= rect[4 * i + 2]; ++a) {
                pr[k].tile = (uint32_t)(b * tx + a);
                pr[k].kappa = s[i].kappa;
                pr[k].idx = i;
                ++k;
            }
    }
    qsort(pr, (size_t)total, sizeof(pair_t), cmp_pair);
    for (int t = 0; t < tx * ty; ++t) tile_start[t] = tile_end[t] = 0;
    for (int64_t j = 0; j < total; ++j) {
        pair_tile[j] = pr[j].tile;
        pair_surf[j] = (uint32_t)pr[j].idx;
        if (j == 0 || pr[j - 1].tile != pr[j].tile) tile_start[pr[j].tile] = (uint32_t)j;
        if (j == total - 1 || pr[j + 1].tile != pr[j].tile) tile_end[pr[j].tile] = (uint32_t)(j + 1);
    }
    if (pair_reached) {
#pragma omp parallel for schedule(dynamic, 256)
        for (int64_t j = 0; j < total; ++j)
            pair_reached[j] = (uint8_t)tile_reached(&s[pr[j].idx], pp, (int)(pr[j].tile % (uint32_t)tx),
                                                    (int)(pr[j].tile / (uint32_t)tx), tile_w, tile_h, W, H);
    }
    free(pr);
    free(s);
    return 0;
}

/* Per-surfel cull/visibility summary for tests: valid flag, fp64 depth,
 * camera-facing normal sign and exact pixel bbox. */
int orc_project(int n, const float *mean, const float *quat, const float *scale, const float *opacity,
                const float *color, int W, int H, const float *intr, const float *viewmat,
                const orc_params *pp, int32_t *valid, double *depth, int32_t *pix_bbox)
{
    for (int i = 0; i < n; ++i) {
        surf_t s;
        preprocess(i, n, mean, quat, scale, opacity, color, W, H, intr, viewmat, pp, &s);
        valid[i] = s.valid;
        depth[i] = s.valid ? s.z : 0.0;
        pix_bbox[4 * i] = s.px0; pix_bbox[4 * i + 1] = s.py0;
        pix_bbox[4 * i + 2] = s.px1; pix_bbox[4 * i + 3] = s.py1;
    }
    return 0;
}
