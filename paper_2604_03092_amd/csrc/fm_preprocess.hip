// fm_preprocess.hip -- per-(view, surfel) projection (forward) and the
// projection chain rule (backward) of the 2DGS rasterizer on gfx950.
//
// Forward: each thread projects one surfel into one view.  The cull
// decisions, the depth key and the pixel bbox are evaluated in FP64 with a
// fixed operation order and no contraction, so that they are bit-identical to
// any other FP64 evaluation of the same formulas in the same order; the
// record the blend kernels read is rounded to FP32.  This is the projection
// of the surfel planar disk (Sec. 3) through the pinhole camera: the local
// plane coordinates (u, v) map to the image by H = K [s_u t_u | s_v t_v | p].
//
// Backward: one thread per surfel walks the views of its submap and chains
// dL/dH, dL/dsigma, dL/dc, dL/dn back to mean, quaternion, scales, opacity,
// colour and the view matrix.  No atomics: each surfel is owned by one
// thread; pose partials are reduced per block and summed by a second kernel.
#include <cstring>

#include "fm_internal.h"
#include "fm_wave.h"

namespace fm {

namespace {

constexpr int kViewChunk = 32;
constexpr int kSubChunk = 32;
constexpr int kListChunk = 512;

struct ViewChunk {
    ViewDesc d[kViewChunk];
    int count, first;
};
struct SubChunk {
    SubmapDesc d[kSubChunk];
    int count, first;
};
struct ListChunk {
    int32_t d[kListChunk];
    int count, first;
};

// Batches of up to 16 views over up to 8 submaps (the common case) travel in
// one launch.
constexpr int kSmallViews = 16;
constexpr int kSmallSubs = 8;
struct SmallSetup {
    ViewDesc v[kSmallViews];
    SubmapDesc s[kSmallSubs];
    int32_t l[kSmallViews];
    int nv, ns;
};
static_assert(sizeof(SmallSetup) <= 4096, "kernel arguments are limited to 4 KB");

// Block 0 writes the descriptors; with `init` the whole grid also starts the
// call's binning state (init_ranges_block).
__global__ __launch_bounds__(256) void k_write_small(SmallSetup c, ViewDesc *ov, SubmapDesc *os, int32_t *ol,
                                                      int init, uint32_t *status, int n_status, uint32_t *tbucket,
                                                      uint32_t *ts, uint32_t *te, int64_t n_tiles) {
    const int i = threadIdx.x;
    if (blockIdx.x == 0) {
        if (i < c.nv) {
            ov[i] = c.v[i];
            ol[i] = c.l[i];
        }
        if (i < c.ns) os[i] = c.s[i];
    }
    if (init) init_ranges_block(status, n_status, tbucket, ts, te, n_tiles);
}

__global__ void k_write_views(ViewChunk c, ViewDesc *out) {
    int i = threadIdx.x;
    if (i < c.count) out[c.first + i] = c.d[i];
}
__global__ void k_write_subs(SubChunk c, SubmapDesc *out) {
    int i = threadIdx.x;
    if (i < c.count) out[c.first + i] = c.d[i];
}
__global__ void k_write_list(ListChunk c, int32_t *out) {
    for (int i = threadIdx.x; i < c.count; i += blockDim.x) out[c.first + i] = c.d[i];
}

// ---------------------------------------------------------------------------
// forward projection
// ---------------------------------------------------------------------------
// Threads take one surfel and up to kProjViews views of its submap: the
// per-surfel part (inputs, finiteness, the normalised quaternion's matrix in
// FP64) is evaluated once for those views.  Block b of the grid belongs to
// the submap whose proj_block_base is the last <= b; within it, blocks run
// over the surfel blocks of 256 for each group of kProjViews views.
constexpr int kProjViews = kProjViewsPerThread;

__device__ inline int submap_of_proj_block(const SubmapDesc *s, int S, int b) {
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (s[mid].proj_block_base <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_preprocess(const SubmapDesc *__restrict__ subs, int S,
                                                     const int32_t *__restrict__ vlist,
                                                     const ViewDesc *__restrict__ views,
                                                     const float *__restrict__ intr,
                                                     const float *__restrict__ viewmat, KParams kp,
                                                     Rec *__restrict__ rec, uint32_t *__restrict__ key,
                                                     uint32_t *__restrict__ cnt, float4 *__restrict__ grad,
                                                     Ell *__restrict__ ell, uint32_t *__restrict__ emeta) {
#pragma clang fp contract(off)
    const SubmapDesc &sd = subs[submap_of_proj_block(subs, S, blockIdx.x)];
    const int n = sd.n;
    const int nsb = (n + 255) >> 8;
    const int lb = (int)blockIdx.x - sd.proj_block_base;
    const int grp = lb / nsb;
    const int i = (lb - grp * nsb) * 256 + (int)threadIdx.x;
    // per surfel
    float f_sig = 0.f, f_c0 = 0.f, f_c1 = 0.f, f_c2 = 0.f;
    double mx = 0.0, my = 0.0, mz = 0.0, su = 0.0, sv = 0.0, sigma = 0.0;
    double Rs[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool sok = false;
    if (i < n) {
        const float f_mx = sd.mean[i], f_my = sd.mean[n + i], f_mz = sd.mean[2 * n + i];
        const float f_qw = sd.quat[i], f_qx = sd.quat[n + i], f_qy = sd.quat[2 * n + i],
                    f_qz = sd.quat[3 * n + i];
        const float f_su = sd.scale[i], f_sv = sd.scale[n + i];
        f_sig = sd.opacity[i];
        f_c0 = sd.color[i]; f_c1 = sd.color[n + i]; f_c2 = sd.color[2 * n + i];
        bool ok = isfinite(f_mx) && isfinite(f_my) && isfinite(f_mz) && isfinite(f_qw) &&
                  isfinite(f_qx) && isfinite(f_qy) && isfinite(f_qz) && isfinite(f_su) &&
                  isfinite(f_sv) && isfinite(f_sig) && isfinite(f_c0) && isfinite(f_c1) &&
                  isfinite(f_c2);
        mx = f_mx; my = f_my; mz = f_mz;
        const double qw = f_qw, qx = f_qx, qy = f_qy, qz = f_qz;
        su = f_su; sv = f_sv; sigma = f_sig;
        ok = ok && (su > 0.0) && (sv > 0.0);
        const double qn = qw * qw + qx * qx + qy * qy + qz * qz;
        ok = ok && (qn > 0.0);
        if (ok) {
            const double qnorm = sqrt(qn);
            const double w = qw / qnorm, x = qx / qnorm, y = qy / qnorm, z = qz / qnorm;
            Rs[0] = 1.0 - 2.0 * (y * y + z * z);
            Rs[1] = 2.0 * (x * y - w * z);
            Rs[2] = 2.0 * (x * z + w * y);
            Rs[3] = 2.0 * (x * y + w * z);
            Rs[4] = 1.0 - 2.0 * (x * x + z * z);
            Rs[5] = 2.0 * (y * z - w * x);
            Rs[6] = 2.0 * (x * z - w * y);
            Rs[7] = 2.0 * (y * z + w * x);
            Rs[8] = 1.0 - 2.0 * (x * x + y * y);
        }
        sok = ok;
    }
    // per view of the group
    const int k_end = min(sd.view_count, (grp + 1) * kProjViews);
    for (int k = grp * kProjViews; k < k_end; ++k) {
        const int v = vlist[sd.view_begin + k];
        const ViewDesc &vd = views[v];
        const int64_t e = (int64_t)vd.entry_base + i;
        uint32_t out_key = 0xFFFFFFFFu, out_cnt = 0;
        bool ok = sok;
        if (ok) {
            const float *vm = viewmat + 12 * v;
            const double R[9] = {vm[0], vm[1], vm[2], vm[4], vm[5], vm[6], vm[8], vm[9], vm[10]};
            const double t[3] = {vm[3], vm[7], vm[11]};
            double p[3], tu[3], tv[3], n0[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                p[r] = R[3 * r] * mx + R[3 * r + 1] * my + R[3 * r + 2] * mz + t[r];
                tu[r] = R[3 * r] * Rs[0] + R[3 * r + 1] * Rs[3] + R[3 * r + 2] * Rs[6];
                tv[r] = R[3 * r] * Rs[1] + R[3 * r + 1] * Rs[4] + R[3 * r + 2] * Rs[7];
                n0[r] = R[3 * r] * Rs[2] + R[3 * r + 1] * Rs[5] + R[3 * r + 2] * Rs[8];
            }
            const double depth = p[2];
            ok = (depth > (double)kp.near_plane) && (sigma > (double)kp.alpha_min);
            if (ok) {
                const float *K = intr + 4 * v;
                const double fx = K[0], fy = K[1], cx = K[2], cy = K[3];
                double M[9];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    M[3 * r + 0] = su * tu[r];
                    M[3 * r + 1] = sv * tv[r];
                    M[3 * r + 2] = p[r];
                }
                double H[9];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    H[c] = fx * M[c] + cx * M[6 + c];
                    H[3 + c] = fy * M[3 + c] + cy * M[6 + c];
                    H[6 + c] = M[6 + c];
                }
                const double rho2 = (double)kp.rho_max * (double)kp.rho_max;
                const double C00 = rho2 * (H[0] * H[0] + H[1] * H[1]) - H[2] * H[2];
                const double C02 = rho2 * (H[0] * H[6] + H[1] * H[7]) - H[2] * H[8];
                const double C11 = rho2 * (H[3] * H[3] + H[4] * H[4]) - H[5] * H[5];
                const double C12 = rho2 * (H[3] * H[6] + H[4] * H[7]) - H[5] * H[8];
                const double C22 = rho2 * (H[6] * H[6] + H[7] * H[7]) - H[8] * H[8];
                const double dx = C02 * C02 - C00 * C22;
                const double dy = C12 * C12 - C11 * C22;
                ok = (C22 < 0.0) && (dx >= 0.0) && (dy >= 0.0);
                if (ok) {
                    const double sx = sqrt(dx), sy = sqrt(dy);
                    const double xa = (C02 - sx) / C22, xb = (C02 + sx) / C22;
                    const double ya = (C12 - sy) / C22, yb = (C12 + sy) / C22;
                    const double xlo = xa < xb ? xa : xb, xhi = xa < xb ? xb : xa;
                    const double ylo = ya < yb ? ya : yb, yhi = ya < yb ? yb : ya;
                    double c0 = ceil(xlo - 0.5), c1 = floor(xhi - 0.5);
                    double r0 = ceil(ylo - 0.5), r1 = floor(yhi - 0.5);
                    if (c0 < 0.0) c0 = 0.0;
                    if (r0 < 0.0) r0 = 0.0;
                    if (c1 > (double)(vd.width - 1)) c1 = (double)(vd.width - 1);
                    if (r1 > (double)(vd.height - 1)) r1 = (double)(vd.height - 1);
                    if (c0 <= c1 && r0 <= r1) {
                        const int px0 = (int)c0, px1 = (int)c1, py0 = (int)r0, py1 = (int)r1;
                        const double dotnp = n0[0] * p[0] + n0[1] * p[1] + n0[2] * p[2];
                        const double sgn = dotnp < 0.0 ? 1.0 : -1.0;
                        const int ixc = (px0 + px1) >> 1, iyc = (py0 + py1) >> 1;
                        const double xs = (double)ixc, ys = (double)iyc;
                        // rows in the shifted pixel frame and the linear ray-plane form
                        const double r0[3] = {H[0] - xs * H[6], H[1] - xs * H[7], H[2] - xs * H[8]};
                        const double r1[3] = {H[3] - ys * H[6], H[4] - ys * H[7], H[5] - ys * H[8]};
                        const double r2[3] = {H[6], H[7], H[8]};
                        const double cc[9] = {r0[1] * r1[2] - r0[2] * r1[1], r0[2] * r1[0] - r0[0] * r1[2],
                                              r0[0] * r1[1] - r0[1] * r1[0], r0[1] * r2[2] - r0[2] * r2[1],
                                              r0[2] * r2[0] - r0[0] * r2[2], r0[0] * r2[1] - r0[1] * r2[0],
                                              r1[1] * r2[2] - r1[2] * r2[1], r1[2] * r2[0] - r1[0] * r2[2],
                                              r1[0] * r2[1] - r1[1] * r2[0]};
                        // a surfel whose plane coefficients exceed 1e30 (a degenerate,
                        // astronomically large projection) is culled, so that every
                        // record's w = c0 + x' c2 - y' c1 is finite over the image
                        bool fin = true;
#pragma unroll
                        for (int k = 0; k < 9; ++k) fin = fin && fabs(cc[k]) <= 1e30;
                        if (fin) {
                            Rec r;
                            r.c0[0] = (float)cc[0]; r.c0[1] = (float)cc[1]; r.c0[2] = (float)cc[2];
                            r.c1[0] = (float)cc[3]; r.c1[1] = (float)cc[4]; r.c1[2] = (float)cc[5];
                            r.c2[0] = (float)cc[6]; r.c2[1] = (float)cc[7]; r.c2[2] = (float)cc[8];
                            r.sigma = f_sig;
                            r.col[0] = f_c0; r.col[1] = f_c1; r.col[2] = f_c2;
                            r.nrm[0] = (float)(sgn * n0[0]);
                            r.nrm[1] = (float)(sgn * n0[1]);
                            r.nrm[2] = (float)(sgn * n0[2]);
                            r.z = (float)depth;
                            r.xs = (float)ixc;
                            r.ys = (float)iyc;
                            // log2(sigma) in FP32: the blend's exponent (one ulp moves sigma G by
                            // < 1e-6 relative; no integer decision depends on it)
                            r.lsig = __log2f(f_sig);
                            // culling ellipse: support radius with the opacity cut-off,
                            // rho_eff^2 = min(rho_max^2, 2 ln(sigma / alpha_min)), enlarged
                            // by 0.2% so that it contains every pixel the FP32 blend accepts
                            {
                                // 2 ln(sigma / alpha_min) in FP32 (its rounding is far inside the
                                // 0.2% enlargement)
                                double re2 = (double)(2.f * (__logf(f_sig) - __logf(kp.alpha_min)));
                                if (re2 > rho2) re2 = rho2;
                                const double E00 = re2 * (H[0] * H[0] + H[1] * H[1]) - H[2] * H[2];
                                const double E01 = re2 * (H[0] * H[3] + H[1] * H[4]) - H[2] * H[5];
                                const double E02 = re2 * (H[0] * H[6] + H[1] * H[7]) - H[2] * H[8];
                                const double E11 = re2 * (H[3] * H[3] + H[4] * H[4]) - H[5] * H[5];
                                const double E12 = re2 * (H[3] * H[6] + H[4] * H[7]) - H[5] * H[8];
                                const double E22 = re2 * (H[6] * H[6] + H[7] * H[7]) - H[8] * H[8];
                                const double i22 = 1.0 / E22, k = 1.002 * i22 * i22;
                                // shape in FP64, the derived slice form in FP32 (the
                                // enlargement above dwarfs its rounding)
                                const double s00 = (E02 * E02 - E00 * E22) * k;
                                const double s01 = (E02 * E12 - E01 * E22) * k;
                                const double s11 = (E12 * E12 - E11 * E22) * k;
                                const float f00 = (float)s00, f01 = (float)s01, f11 = (float)s11;
                                const float fdet = (float)(s00 * s11 - s01 * s01);
                                Ell el;
                                el.ex = (float)(E02 * i22);
                                el.ey = (float)(E12 * i22);
                                el.hx = f00 > 0.f ? sqrtf(f00) : 0.f;
                                el.hy = f11 > 0.f ? sqrtf(f11) : 0.f;
                                el.k1 = f11 > 0.f ? f01 / f11 : 0.f;
                                el.k2 = f11 > 0.f && fdet > 0.f ? (fdet / f11) / f11 : 0.f;
                                el.dyr = el.hx > 0.f ? f01 / el.hx : 0.f;
                                for (int k = 0; k < 6; ++k) el.pad[k] = 0u;
                                const int tx0 = px0 / kp.tile_w, tx1 = px1 / kp.tile_w;
                                const int ty0 = py0 / kp.tile_h;
                                el.tb = (uint32_t)(vd.tile_base + ty0 * vd.tiles_x + tx0);
                                el.t0 = (uint32_t)tx0 | ((uint32_t)ty0 << 16);
                                el.nt = (uint32_t)(tx1 - tx0 + 1) | ((uint32_t)vd.tiles_x << 16);
                                ell[e] = el;
                            }
                            rec[e] = r;
                            // what the backward projection needs of the record: the
                            // pixel-frame shift and whether the normal was flipped
                            emeta[e] = (uint32_t)ixc | ((uint32_t)iyc << 14) | (sgn < 0.0 ? 0x80000000u : 0u);
                            const int tx0 = px0 / kp.tile_w, tx1 = px1 / kp.tile_w;
                            const int ty0 = py0 / kp.tile_h, ty1 = py1 / kp.tile_h;
                            out_cnt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
                            out_key = __float_as_uint((float)depth);
                        }
                    }
                }
            }
        }
        key[e] = out_key;
        cnt[e] = out_cnt;
        if (grad && out_cnt != 0) {  // the fused path clears the entry's gradient slot here
            const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
            const int q = kp.gstride / 4;
            for (int kk = 0; kk < q; ++kk) grad[q * e + kk] = z;
        }
    }
}

// Zero the gradient slot (gstride floats) of every entry that has pairs.
__global__ __launch_bounds__(256) void k_zero_grad(const uint32_t *__restrict__ cnt, float4 *__restrict__ grad,
                                                    int64_t E, int gstride) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < E && cnt[e] != 0) {
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        const int q = gstride / 4;
        for (int k = 0; k < q; ++k) grad[q * e + k] = z;
    }
}

// ---------------------------------------------------------------------------
// backward projection (one thread per surfel, looping over its views)
// ---------------------------------------------------------------------------
__device__ inline int submap_of_block(const SubmapDesc *s, int S, int b) {
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (s[mid].block_base <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Pruning scores: one thread per surfel of a rendered submap sums its
// entries' scores (the first float of each gradient slot of an entry with
// pairs) over the submap's views in view order and stores the sum into the
// submap's g_opacity plane, which the pruning call points at the caller's
// score array.
__global__ __launch_bounds__(256) void k_score_reduce(const SubmapDesc *__restrict__ subs, int S,
                                                       const int32_t *__restrict__ vlist,
                                                       const ViewDesc *__restrict__ views,
                                                       const uint32_t *__restrict__ cnt,
                                                       const float *__restrict__ grad, int gstride) {
    const SubmapDesc &sd = subs[submap_of_block(subs, S, blockIdx.x)];
    const int i = ((int)blockIdx.x - sd.block_base) * 256 + (int)threadIdx.x;
    if (i >= sd.n || !sd.g_opacity) return;
    float sc = 0.f;
    for (int k = 0; k < sd.view_count; ++k) {
        const int64_t e = (int64_t)views[vlist[sd.view_begin + k]].entry_base + i;
        if (cnt[e] != 0) sc += grad[e * gstride];
    }
    sd.g_opacity[i] = sc;
}

__global__ __launch_bounds__(256) void k_preprocess_bwd(
    const SubmapDesc *__restrict__ subs, int S, const int32_t *__restrict__ vlist,
    const ViewDesc *__restrict__ views, const float *__restrict__ intr,
    const float *__restrict__ viewmat, const uint32_t *__restrict__ emeta, const uint32_t *__restrict__ cnt,
    const float4 *__restrict__ grad, int gstride, float *__restrict__ pose_part, int max_blocks,
    int overwrite) {
    const int s_idx = submap_of_block(subs, S, blockIdx.x);
    const SubmapDesc &sd = subs[s_idx];
    const int lb = blockIdx.x - sd.block_base;
    const int i = lb * 256 + threadIdx.x;
    const int n = sd.n;
    const bool live = i < n;
    const int wave = threadIdx.x >> 6;

    float mu[3] = {0.f, 0.f, 0.f}, qh[4] = {1.f, 0.f, 0.f, 0.f}, qnorm = 1.f, su = 0.f, sv = 0.f;
    float Rs[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
    if (live) {
        mu[0] = sd.mean[i]; mu[1] = sd.mean[n + i]; mu[2] = sd.mean[2 * n + i];
        const float q0 = sd.quat[i], q1 = sd.quat[n + i], q2 = sd.quat[2 * n + i], q3 = sd.quat[3 * n + i];
        su = sd.scale[i]; sv = sd.scale[n + i];
        const float qn = q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3;
        if (qn > 0.f && isfinite(qn)) {
            qnorm = sqrtf(qn);
            const float inv = 1.f / qnorm;
            qh[0] = q0 * inv; qh[1] = q1 * inv; qh[2] = q2 * inv; qh[3] = q3 * inv;
        }
        const float w = qh[0], x = qh[1], y = qh[2], z = qh[3];
        Rs[0] = 1.f - 2.f * (y * y + z * z);
        Rs[1] = 2.f * (x * y - w * z);
        Rs[2] = 2.f * (x * z + w * y);
        Rs[3] = 2.f * (x * y + w * z);
        Rs[4] = 1.f - 2.f * (x * x + z * z);
        Rs[5] = 2.f * (y * z - w * x);
        Rs[6] = 2.f * (x * z - w * y);
        Rs[7] = 2.f * (y * z + w * x);
        Rs[8] = 1.f - 2.f * (x * x + y * y);
    }
    float dmu[3] = {0.f, 0.f, 0.f}, dRs[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float dsu = 0.f, dsv = 0.f, dsig = 0.f, dc[3] = {0.f, 0.f, 0.f};

    for (int k = 0; k < sd.view_count; ++k) {
        const int v = vlist[sd.view_begin + k];
        const ViewDesc &vd = views[v];
        const int64_t e = (int64_t)vd.entry_base + i;
        float dV[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) dV[j] = 0.f;
        if (live && cnt[e] != 0) {
            const float4 *gp = grad + (gstride / 4) * e;
            // without normal gradients the slot ends after component 15
            const float4 g4 = gstride > kGradSlot ? gp[4] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float4 g0 = gp[0], g1 = gp[1], g2 = gp[2], g3 = gp[3];
            const float g[20] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w, g2.x, g2.y,
                                 g2.z, g2.w, g3.x, g3.y, g3.z, g3.w, g4.x, g4.y, g4.z, g4.w};
            const uint32_t em = emeta[e];
            const float xs = (float)(em & 0x3FFFu), ys = (float)((em >> 14) & 0x3FFFu);
            const float *vm = viewmat + 12 * v;
            const float R[9] = {vm[0], vm[1], vm[2], vm[4], vm[5], vm[6], vm[8], vm[9], vm[10]};
            const float *K = intr + 4 * v;
            const float fx = K[0], fy = K[1], cx = K[2], cy = K[3];
            const float ox = cx - xs, oy = cy - ys;
            // The camera-frame tangents and centre and the shifted rows
            // r0 = fx M0 + (cx - xs) M2, r1 = fy M1 + (cy - ys) M2, r2 = M2 of
            // M = [s_u t_u | s_v t_v | p] are formed in FP64: the shift cancels
            // most of fx p0 and fy p1, and for surfels seen at grazing angles
            // the FP32 rounding of p, amplified by that cancellation, reached
            // 1e-3 of the gradients' rms.  The rest of the chain is FP32.
            float tu[3], tv[3], n0[3], r0[3], r1[3], r2[3];
            // column c of M: s_u t_u, s_v t_v, p (one column's three doubles at a time)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double m[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const double a = R[3 * r], b = R[3 * r + 1], e = R[3 * r + 2];
                    if (c < 2) {
                        const double x = a * Rs[c] + b * Rs[3 + c] + e * Rs[6 + c];
                        if (c == 0) tu[r] = (float)x; else tv[r] = (float)x;
                        m[r] = (c == 0 ? (double)su : (double)sv) * x;
                    } else {
                        m[r] = a * mu[0] + b * mu[1] + e * mu[2] + (double)vm[4 * r + 3];
                    }
                }
                r0[c] = (float)((double)fx * m[0] + (double)ox * m[2]);
                r1[c] = (float)((double)fy * m[1] + (double)oy * m[2]);
                r2[c] = (float)m[2];
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) n0[r] = R[3 * r] * Rs[2] + R[3 * r + 1] * Rs[5] + R[3 * r + 2] * Rs[8];
            // c0 = r0 x r1, c1 = r0 x r2, c2 = r1 x r2  ->  d(r0, r1, r2)
            const float dc0[3] = {g[0], g[1], g[2]}, dc1[3] = {g[3], g[4], g[5]}, dc2[3] = {g[6], g[7], g[8]};
            float dr0[3], dr1[3], dr2[3];
            dr0[0] = (r1[1] * dc0[2] - r1[2] * dc0[1]) + (r2[1] * dc1[2] - r2[2] * dc1[1]);
            dr0[1] = (r1[2] * dc0[0] - r1[0] * dc0[2]) + (r2[2] * dc1[0] - r2[0] * dc1[2]);
            dr0[2] = (r1[0] * dc0[1] - r1[1] * dc0[0]) + (r2[0] * dc1[1] - r2[1] * dc1[0]);
            dr1[0] = (dc0[1] * r0[2] - dc0[2] * r0[1]) + (r2[1] * dc2[2] - r2[2] * dc2[1]);
            dr1[1] = (dc0[2] * r0[0] - dc0[0] * r0[2]) + (r2[2] * dc2[0] - r2[0] * dc2[2]);
            dr1[2] = (dc0[0] * r0[1] - dc0[1] * r0[0]) + (r2[0] * dc2[1] - r2[1] * dc2[0]);
            dr2[0] = (dc1[1] * r0[2] - dc1[2] * r0[1]) + (dc2[1] * r1[2] - dc2[2] * r1[1]);
            dr2[1] = (dc1[2] * r0[0] - dc1[0] * r0[2]) + (dc2[2] * r1[0] - dc2[0] * r1[2]);
            dr2[2] = (dc1[0] * r0[1] - dc1[1] * r0[0]) + (dc2[0] * r1[1] - dc2[1] * r1[0]);
            // r0 = fx M0 + (cx - xs) M2, r1 = fy M1 + (cy - ys) M2, r2 = M2  ->  dM
            float dM[9];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dM[c] = fx * dr0[c];
                dM[3 + c] = fy * dr1[c];
                dM[6 + c] = ox * dr0[c] + oy * dr1[c] + dr2[c];
            }
            const float sgn = (em & 0x80000000u) ? -1.f : 1.f;  // the projection's camera-facing flip
            const float dp[3] = {dM[2], dM[5], dM[8] + g[13]};
            const float dtu[3] = {su * dM[0], su * dM[3], su * dM[6]};
            const float dtv[3] = {sv * dM[1], sv * dM[4], sv * dM[7]};
            dsu += tu[0] * dM[0] + tu[1] * dM[3] + tu[2] * dM[6];
            dsv += tv[0] * dM[1] + tv[1] * dM[4] + tv[2] * dM[7];
            const float dn0[3] = {sgn * g[14], sgn * g[15], sgn * g[16]};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                dmu[c] += R[c] * dp[0] + R[3 + c] * dp[1] + R[6 + c] * dp[2];
                dRs[3 * c + 0] += R[c] * dtu[0] + R[3 + c] * dtu[1] + R[6 + c] * dtu[2];
                dRs[3 * c + 1] += R[c] * dtv[0] + R[3 + c] * dtv[1] + R[6 + c] * dtv[2];
                dRs[3 * c + 2] += R[c] * dn0[0] + R[3 + c] * dn0[1] + R[6 + c] * dn0[2];
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    dV[4 * r + c] = dp[r] * mu[c] + dtu[r] * Rs[3 * c] + dtv[r] * Rs[3 * c + 1] +
                                    dn0[r] * Rs[3 * c + 2];
                dV[4 * r + 3] = dp[r];
            }
            dsig += g[9];
            dc[0] += g[10]; dc[1] += g[11]; dc[2] += g[12];
        }
        // wave reduction of the 12 pose-gradient values of view v into this
        // wave's partial (no block barrier: the waves run the views at their own pace)
        const float r = wave_reduce16(dV);
        const int comp = wave_reduce16_component();
        if (comp >= 0 && comp < 12) pose_part[(((int64_t)v * max_blocks + lb) * 4 + wave) * 12 + comp] = r;
    }
    if (!live) return;
    // dL/d(unit quaternion) from dL/dR_s, then project onto the raw quaternion
    const float w = qh[0], x = qh[1], y = qh[2], z = qh[3];
    const float *G = dRs;
    float dq[4];
    dq[0] = 2.f * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
    dq[1] = 2.f * (y * G[1] + z * G[2] + y * G[3] - 2.f * x * G[4] - w * G[5] + z * G[6] + w * G[7] -
                   2.f * x * G[8]);
    dq[2] = 2.f * (-2.f * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] -
                   2.f * y * G[8]);
    dq[3] = 2.f * (-2.f * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.f * z * G[4] + y * G[5] +
                   x * G[6] + y * G[7]);
    const float dot = dq[0] * w + dq[1] * x + dq[2] * y + dq[3] * z;
    const float inv = 1.f / qnorm;
    // add into the caller's gradients, or store them (overwrite)
    const bool ow = overwrite != 0;
    auto put = [ow](float *g, float v) { *g = ow ? v : *g + v; };
    if (sd.g_mean) {
        put(sd.g_mean + i, dmu[0]);
        put(sd.g_mean + n + i, dmu[1]);
        put(sd.g_mean + 2 * n + i, dmu[2]);
    }
    if (sd.g_quat) {
        put(sd.g_quat + i, (dq[0] - w * dot) * inv);
        put(sd.g_quat + n + i, (dq[1] - x * dot) * inv);
        put(sd.g_quat + 2 * n + i, (dq[2] - y * dot) * inv);
        put(sd.g_quat + 3 * n + i, (dq[3] - z * dot) * inv);
    }
    if (sd.g_scale) {
        put(sd.g_scale + i, dsu);
        put(sd.g_scale + n + i, dsv);
    }
    if (sd.g_opacity) put(sd.g_opacity + i, dsig);
    if (sd.g_color) {
        put(sd.g_color + i, dc[0]);
        put(sd.g_color + n + i, dc[1]);
        put(sd.g_color + 2 * n + i, dc[2]);
    }
}

// dL_dviewmat[v] += sum over the blocks of v's submap of the pose partials.
__global__ __launch_bounds__(1024) void k_pose_reduce(const ViewDesc *__restrict__ views,
                                                       const SubmapDesc *__restrict__ subs,
                                                       const float *__restrict__ pose_part, int max_blocks,
                                                       float *__restrict__ dL_dviewmat, int overwrite) {
    __shared__ float red[16][16];
    const int v = blockIdx.x;
    const SubmapDesc &sd = subs[views[v].submap];
    const int nw = 4 * ((sd.n + 255) / 256);  // one partial per wave of the submap's blocks
    float acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.f;
    const float4 *base = reinterpret_cast<const float4 *>(pose_part + (int64_t)v * max_blocks * 4 * 12);
    for (int b = threadIdx.x; b < nw; b += 1024) {
        const float4 x = base[3 * b], y = base[3 * b + 1], z = base[3 * b + 2];
        acc[0] += x.x; acc[1] += x.y; acc[2] += x.z; acc[3] += x.w;
        acc[4] += y.x; acc[5] += y.y; acc[6] += y.z; acc[7] += y.w;
        acc[8] += z.x; acc[9] += z.y; acc[10] += z.z; acc[11] += z.w;
    }
    const float r = wave_reduce16(acc);
    const int comp = wave_reduce16_component();
    if (comp >= 0) red[threadIdx.x >> 6][comp] = r;
    __syncthreads();
    if (threadIdx.x < 12) {
        float t = 0.f;
        for (int w = 0; w < 16; ++w) t += red[w][threadIdx.x];
        float *d = dL_dviewmat + 12 * v + threadIdx.x;
        *d = overwrite ? t : *d + t;
    }
}

}  // namespace

hipError_t launch_setup(const Plan &p, void *ws, const ViewDesc *views, const SubmapDesc *subs,
                        const int32_t *vlist, bool start_binning, hipStream_t st) {
    if (p.V <= kSmallViews && p.S <= kSmallSubs) {
        SmallSetup c;
        memset(&c, 0, sizeof(c));
        c.nv = p.V;
        c.ns = p.S;
        for (int i = 0; i < p.V; ++i) {
            c.v[i] = views[i];
            c.l[i] = vlist[i];
        }
        for (int i = 0; i < p.S; ++i) c.s[i] = subs[i];
        static_assert(kSmallViews <= 256 && kSmallSubs <= 256, "one thread per descriptor");
        hipLaunchKernelGGL(k_write_small, dim3(start_binning ? init_ranges_blocks(p) : 1), dim3(256), 0, st, c,
                           at<ViewDesc>(ws, p.o_views), at<SubmapDesc>(ws, p.o_subs), at<int32_t>(ws, p.o_vlist),
                           start_binning ? 1 : 0,
                           reinterpret_cast<uint32_t *>(at<Status>(ws, p.o_status)), (int)(sizeof(Status) / 4),
                           at<uint32_t>(ws, p.o_tbucket), at<uint32_t>(ws, p.o_tstart), at<uint32_t>(ws, p.o_tend),
                           p.T);
        return hipGetLastError();
    }
    if (start_binning) {
        const hipError_t e = launch_init_ranges(p, ws, st);
        if (e != hipSuccess) return e;
    }
    for (int f = 0; f < p.V; f += kViewChunk) {
        ViewChunk c;
        c.first = f;
        c.count = p.V - f < kViewChunk ? p.V - f : kViewChunk;
        for (int i = 0; i < c.count; ++i) c.d[i] = views[f + i];
        hipLaunchKernelGGL(k_write_views, dim3(1), dim3(kViewChunk), 0, st, c, at<ViewDesc>(ws, p.o_views));
    }
    for (int f = 0; f < p.S; f += kSubChunk) {
        SubChunk c;
        c.first = f;
        c.count = p.S - f < kSubChunk ? p.S - f : kSubChunk;
        for (int i = 0; i < c.count; ++i) c.d[i] = subs[f + i];
        hipLaunchKernelGGL(k_write_subs, dim3(1), dim3(kSubChunk), 0, st, c, at<SubmapDesc>(ws, p.o_subs));
    }
    for (int f = 0; f < p.V; f += kListChunk) {
        ListChunk c;
        c.first = f;
        c.count = p.V - f < kListChunk ? p.V - f : kListChunk;
        for (int i = 0; i < c.count; ++i) c.d[i] = vlist[f + i];
        hipLaunchKernelGGL(k_write_list, dim3(1), dim3(256), 0, st, c, at<int32_t>(ws, p.o_vlist));
    }
    return hipGetLastError();
}

hipError_t launch_preprocess(const Plan &p, void *ws, const KParams &kp, const float *intr,
                             const float *viewmat, bool zero_grad, hipStream_t st) {
    if (p.proj_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_preprocess, dim3(p.proj_blocks), dim3(256), 0, st, at<SubmapDesc>(ws, p.o_subs), p.S,
                       at<int32_t>(ws, p.o_vlist), at<ViewDesc>(ws, p.o_views),
                       intr, viewmat, kp, at<Rec>(ws, p.o_rec), at<uint32_t>(ws, p.o_key),
                       at<uint32_t>(ws, p.o_cnt), zero_grad ? at<float4>(ws, p.o_grad) : nullptr,
                       at<Ell>(ws, p.o_ell), at<uint32_t>(ws, p.o_emeta));
    return hipGetLastError();
}

hipError_t launch_zero_grad(const Plan &p, void *ws, int gstride, hipStream_t st) {
    const int blocks = (int)((p.E + 255) / 256);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_grad, dim3(blocks), dim3(256), 0, st, at<uint32_t>(ws, p.o_cnt),
                       at<float4>(ws, p.o_grad), p.E, gstride);
    return hipGetLastError();
}

hipError_t launch_score_reduce(const Plan &p, void *ws, int gstride, hipStream_t st) {
    if (p.a7_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_score_reduce, dim3(p.a7_blocks), dim3(256), 0, st, at<SubmapDesc>(ws, p.o_subs), p.S,
                       at<int32_t>(ws, p.o_vlist), at<ViewDesc>(ws, p.o_views), at<uint32_t>(ws, p.o_cnt),
                       at<float>(ws, p.o_grad), gstride);
    return hipGetLastError();
}

hipError_t launch_preprocess_bwd(const Plan &p, void *ws, int gstride, const float *intr, const float *viewmat,
                                 float *dL_dviewmat, hipStream_t st) {
    if (p.a7_blocks > 0) {
        hipLaunchKernelGGL(k_preprocess_bwd, dim3(p.a7_blocks), dim3(256), 0, st,
                           at<SubmapDesc>(ws, p.o_subs), p.S, at<int32_t>(ws, p.o_vlist),
                           at<ViewDesc>(ws, p.o_views), intr, viewmat, at<uint32_t>(ws, p.o_emeta),
                           at<uint32_t>(ws, p.o_cnt), at<float4>(ws, p.o_grad), gstride,
                           at<float>(ws, p.o_pose), p.a7_max_blocks, (int)p.overwrite);
    }
    if (dL_dviewmat) {
        hipLaunchKernelGGL(k_pose_reduce, dim3(p.V), dim3(1024), 0, st, at<ViewDesc>(ws, p.o_views),
                           at<SubmapDesc>(ws, p.o_subs), at<float>(ws, p.o_pose), p.a7_max_blocks,
                           dL_dviewmat, (int)p.overwrite);
    }
    return hipGetLastError();
}

}  // namespace fm
