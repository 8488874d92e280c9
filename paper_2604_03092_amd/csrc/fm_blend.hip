// fm_blend.hip -- per-tile front-to-back compositing (Eq. 1) and its adjoint
// on gfx950.
//
// One workgroup per tile; each wave64 owns an 8x8 pixel block of the tile.
// The tile's depth-ordered surfels are staged through LDS in batches of one
// record per thread; every wave reads them as broadcasts and skips a whole
// surfel with one scalar test when the surfel's pixel bbox misses its block.
// Waves stop when all their pixels have reached the transmittance floor.
//
// Backward (forward order, no per-pixel lists): with f_k = g . (c_k, z_k,
// n_k, 1) and S = g . (I, D, N, A) known from the forward outputs, the
// adjoint of the compositing is
//     dL/dalpha_k = T_k f_k - (S - S_k) / (1 - alpha_k),   S_k = sum_{j<=k} f_j alpha_j T_j,
// so the backward walks the list front to back exactly like the forward,
// recomputing T, and stops at the pixel's last contributor.  Per surfel, the
// screen-space gradients of a wave are reduced with permlane swaps + DPP and
// added into the entry's gradient slot with one coalesced 16-float atomic
// group (plus one for the last normal component when normals carry a
// gradient).
#include "fm_internal.h"
#include "fm_wave.h"

namespace fm {

namespace {

struct Surf {
    float c00, c01, c02, c10, c11, c12, c20, c21, c22;
    float sig, r, g, b, n0, n1, n2, z, xs, ys;
};

__device__ __forceinline__ void load_surf(const Rec *rp, Surf &s) {
    const float4 *p = reinterpret_cast<const float4 *>(rp);
    const float4 a = p[0], b = p[1], c = p[2], d = p[3], e = p[4];
    s.c00 = a.x; s.c01 = a.y; s.c02 = a.z; s.c10 = a.w;
    s.c11 = b.x; s.c12 = b.y; s.c20 = b.z; s.c21 = b.w;
    s.c22 = c.x; s.sig = c.y; s.r = c.z; s.g = c.w;
    s.b = d.x; s.n0 = d.y; s.n1 = d.z; s.n2 = d.w;
    s.z = e.x; s.xs = e.y; s.ys = e.z;
}

struct Hit {
    float xp, yp, w0, w1, w2, r2;
    float G, at, alpha;
};

// Ray-splat intersection at the pixel centre (px, py): in the surfel's
// shifted pixel frame, w = c0 + x' c2 - y' c1 and (u, v) = (w0, w1) / w2.
// Returns false when the pixel is outside the rho_max support or
// sigma G < alpha_min.  Identical arithmetic in forward and backward (no
// contraction beyond the explicit fmaf calls), so both see the same decisions.
__device__ __forceinline__ bool splat(const Surf &s, float px, float py, float rho2, float amin, float amax,
                                      Hit &h) {
#pragma clang fp contract(off)
    h.xp = px - s.xs;
    h.yp = py - s.ys;
    h.w0 = fmaf(h.xp, s.c20, fmaf(-h.yp, s.c10, s.c00));
    h.w1 = fmaf(h.xp, s.c21, fmaf(-h.yp, s.c11, s.c01));
    h.w2 = fmaf(h.xp, s.c22, fmaf(-h.yp, s.c12, s.c02));
    const float num = fmaf(h.w0, h.w0, h.w1 * h.w1);
    const float den = h.w2 * h.w2;
    if (!(num <= rho2 * den) || !(den > 0.f)) return false;
    h.r2 = num * __builtin_amdgcn_rcpf(den);
    h.G = __builtin_amdgcn_exp2f(h.r2 * -0.72134752044448170368f);  // exp(-r2/2)
    h.at = s.sig * h.G;
    if (!(h.at >= amin)) return false;
    h.alpha = fminf(amax, h.at);
    return true;
}

template <int TW, int TH> struct Geo {
    static constexpr int NT = TW * TH;
    static constexpr int WX = TW / 8;
    static constexpr int NW = NT / 64;
};

struct PixelCtx {
    int view, col, row, wx0, wy0;
    bool inside;
    int64_t pix;       // global pixel index
    float px, py;
    uint32_t start, end;
    int W, H;
    uint32_t n_entries;
};

template <int TW, int TH>
__device__ __forceinline__ PixelCtx pixel_ctx(const ViewDesc *views, int V, const uint32_t *ts,
                                              const uint32_t *te) {
    using Gm = Geo<TW, TH>;
    PixelCtx c;
    const int tile = blockIdx.x;
    c.view = view_of_tile(views, V, tile);
    const ViewDesc &vd = views[c.view];
    const int local = tile - vd.tile_base;
    const int tx = local % vd.tiles_x, ty = local / vd.tiles_x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    c.wx0 = tx * TW + (wave % Gm::WX) * 8;
    c.wy0 = ty * TH + (wave / Gm::WX) * 8;
    c.col = c.wx0 + (lane & 7);
    c.row = c.wy0 + (lane >> 3);
    c.W = vd.width;
    c.H = vd.height;
    c.inside = c.col < vd.width && c.row < vd.height;
    c.pix = vd.pixel_offset + (int64_t)c.row * vd.width + c.col;
    c.px = (float)c.col + 0.5f;
    c.py = (float)c.row + 0.5f;
    c.start = ts[tile];
    c.end = te[tile];
    // total entries: the last view's segment end
    c.n_entries = (uint32_t)views[V - 1].entry_base + (((uint32_t)views[V - 1].n + 255u) & ~255u);
    return c;
}

// Does the pair's 8x8-block mask exclude this wave's block?  Scalar test.
__device__ __forceinline__ bool block_miss(const uint32_t *sval, int j, int wave) {
    const uint32_t m = __builtin_amdgcn_readfirstlane(sval[j]);
    return ((m >> (kMaskShift + wave)) & 1u) == 0u;
}

// Forward traversal of the tile list.  acc = (r, g, b, depth, nx, ny, nz, A).
template <int TW, int TH>
__device__ __forceinline__ void tile_forward(const PixelCtx &c, const uint32_t *__restrict__ pval,
                                             const Rec *__restrict__ rec, const KParams &kp, Rec *srec,
                                             uint32_t *sval, float acc[8], float &T, uint32_t &nlast,
                                             uint32_t &ncount) {
    using Gm = Geo<TW, TH>;
    const float rho2 = kp.rho_max * kp.rho_max;
    bool done = !c.inside;
    T = 1.f;
    nlast = 0;
    ncount = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.f;
    for (uint32_t base = c.start; base < c.end; base += Gm::NT) {
        if (__syncthreads_count(!done) == 0) break;
        const int cntb = (int)min((uint32_t)Gm::NT, c.end - base);
        if ((int)threadIdx.x < cntb) {
            const uint32_t pv = pval[base + threadIdx.x];
            const bool ok = (pv & kEntryMask) < c.n_entries;  // guards the record load
            sval[threadIdx.x] = ok ? pv : 0u;
            if (ok) srec[threadIdx.x] = rec[pv & kEntryMask];
        }
        __syncthreads();
        if (ballot64(!done) == 0) continue;
        const int wave = threadIdx.x >> 6;
        for (int j = 0; j < cntb; ++j) {
            if (block_miss(sval, j, wave)) continue;
            if (!done) {
                Surf s;
                load_surf(&srec[j], s);
                Hit h;
                if (splat(s, c.px, c.py, rho2, kp.alpha_min, kp.alpha_max, h)) {
#pragma clang fp contract(off)
                    const float test = T * (1.f - h.alpha);
                    if (test < kp.t_min) {
                        done = true;
                    } else {
                        const float wgt = h.alpha * T;
                        acc[0] = fmaf(s.r, wgt, acc[0]);
                        acc[1] = fmaf(s.g, wgt, acc[1]);
                        acc[2] = fmaf(s.b, wgt, acc[2]);
                        acc[3] = fmaf(s.z, wgt, acc[3]);
                        acc[4] = fmaf(s.n0, wgt, acc[4]);
                        acc[5] = fmaf(s.n1, wgt, acc[5]);
                        acc[6] = fmaf(s.n2, wgt, acc[6]);
                        acc[7] = acc[7] + wgt;
                        T = test;
                        nlast = base - c.start + (uint32_t)j + 1u;
                        ++ncount;
                    }
                }
            }
            if (ballot64(!done) == 0) break;
        }
    }
}

// Adjoint traversal.  g = dL/d(r, g, b, depth, nx, ny, nz, A) of this pixel,
// S = g . outputs, nlast = this pixel's contributor prefix length, maxlast =
// the tile's maximum.  HAS_N: the normal map carries a gradient.
// Accumulates into the entries' gradient slots (kGradStride floats each).
template <int TW, int TH, bool HAS_N>
__device__ __forceinline__ void tile_backward(const PixelCtx &c, const uint32_t *__restrict__ pval,
                                              const Rec *__restrict__ rec, const KParams &kp, Rec *srec,
                                              uint32_t *sval, const float g[8], float S, uint32_t nlast,
                                              uint32_t maxlast, float *__restrict__ grad) {
    using Gm = Geo<TW, TH>;
    const float rho2 = kp.rho_max * kp.rho_max;
    float T = 1.f, Sk = 0.f;
    const uint32_t len = c.end - c.start;
    const uint32_t end = c.start + (maxlast < len ? maxlast : len);
    const int comp = wave_reduce16_component();
    for (uint32_t base = c.start; base < end; base += Gm::NT) {
        const int cntb = (int)min((uint32_t)Gm::NT, end - base);
        __syncthreads();
        if ((int)threadIdx.x < cntb) {
            const uint32_t pv = pval[base + threadIdx.x];
            const bool ok = (pv & kEntryMask) < c.n_entries;  // guards the record load
            sval[threadIdx.x] = ok ? pv : 0u;
            if (ok) srec[threadIdx.x] = rec[pv & kEntryMask];
        }
        __syncthreads();
        const uint32_t kbase = base - c.start;
        if (ballot64(kbase < nlast) == 0) continue;
        const int wave = threadIdx.x >> 6;
        for (int j = 0; j < cntb; ++j) {
            if (block_miss(sval, j, wave)) continue;
            const bool live = kbase + (uint32_t)j < nlast;
            if (ballot64(live) == 0) break;
            float gr[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) gr[k] = 0.f;
            float gn2 = 0.f;
            bool hit = false;
            if (live) {
                Surf s;
                load_surf(&srec[j], s);
                Hit h;
                if (splat(s, c.px, c.py, rho2, kp.alpha_min, kp.alpha_max, h)) {
#pragma clang fp contract(off)
                    hit = true;
                    const float test = T * (1.f - h.alpha);
                    const float wgt = h.alpha * T;
                    float f = g[0] * s.r + g[1] * s.g + g[2] * s.b + g[3] * s.z + g[7];
                    if (HAS_N) f += g[4] * s.n0 + g[5] * s.n1 + g[6] * s.n2;
                    Sk = fmaf(f, wgt, Sk);
                    const float dal = T * f - (S - Sk) * __builtin_amdgcn_rcpf(1.f - h.alpha);
                    gr[10] = g[0] * wgt;
                    gr[11] = g[1] * wgt;
                    gr[12] = g[2] * wgt;
                    gr[13] = g[3] * wgt;
                    if (HAS_N) {
                        gr[14] = g[4] * wgt;
                        gr[15] = g[5] * wgt;
                        gn2 = g[6] * wgt;
                    }
                    if (h.at <= kp.alpha_max) {
                        // alpha = sigma G, G = exp(-r2/2), r2 = (w0^2 + w1^2) / w2^2
                        gr[9] = dal * h.G;
                        const float dr2 = -0.5f * h.G * s.sig * dal;
                        const float iw = __builtin_amdgcn_rcpf(h.w2);
                        const float q = 2.f * dr2 * iw;
                        const float gw0 = q * h.w0 * iw, gw1 = q * h.w1 * iw, gw2 = -q * h.r2;
                        // w = c0 + x' c2 - y' c1
                        gr[0] = gw0; gr[1] = gw1; gr[2] = gw2;
                        gr[3] = -h.yp * gw0; gr[4] = -h.yp * gw1; gr[5] = -h.yp * gw2;
                        gr[6] = h.xp * gw0; gr[7] = h.xp * gw1; gr[8] = h.xp * gw2;
                    }
                    T = test;
                }
            }
            if (ballot64(hit) == 0) continue;
            const float r = wave_reduce16(gr);
            float *dst = grad + (int64_t)(sval[j] & kEntryMask) * kGradStride;
            if (comp >= 0) atomicAdd(dst + comp, r);
            if (HAS_N) {
                const float t2 = wave_sum(gn2);
                if (lane_id() == 0) atomicAdd(dst + 16, t2);
            }
        }
    }
}

template <int NT> __device__ __forceinline__ uint32_t block_max(uint32_t v, uint32_t *scratch) {
    if (threadIdx.x == 0) *scratch = 0;
    __syncthreads();
    atomicMax(scratch, v);
    __syncthreads();
    const uint32_t r = *scratch;
    __syncthreads();
    return r;
}

template <int NT> __device__ __forceinline__ float block_sum(float v, float *scratch) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
    __syncthreads();
    float s = 0.f;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k) s += scratch[k];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------------------
template <int TW, int TH>
__global__ __launch_bounds__(TW *TH) void k_render_fwd(const ViewDesc *__restrict__ views, int V,
                                                        const uint32_t *__restrict__ ts,
                                                        const uint32_t *__restrict__ te,
                                                        const uint32_t *__restrict__ pval,
                                                        const Rec *__restrict__ rec, KParams kp, int64_t NPX,
                                                        fm_outputs out, float *__restrict__ tfinal,
                                                        uint32_t *__restrict__ nlast_out,
                                                        uint32_t *__restrict__ ncount_out) {
    using Gm = Geo<TW, TH>;
    __shared__ Rec srec[Gm::NT];
    __shared__ uint32_t sval[Gm::NT];
    const PixelCtx c = pixel_ctx<TW, TH>(views, V, ts, te);
    float acc[8], T;
    uint32_t nl, nc;
    tile_forward<TW, TH>(c, pval, rec, kp, srec, sval, acc, T, nl, nc);
    if (c.inside) {
        out.rgb[c.pix] = acc[0] + T * kp.bg[0];
        out.rgb[NPX + c.pix] = acc[1] + T * kp.bg[1];
        out.rgb[2 * NPX + c.pix] = acc[2] + T * kp.bg[2];
        out.depth[c.pix] = acc[3];
        out.normal[c.pix] = acc[4];
        out.normal[NPX + c.pix] = acc[5];
        out.normal[2 * NPX + c.pix] = acc[6];
        out.alpha[c.pix] = acc[7];
        tfinal[c.pix] = T;
        nlast_out[c.pix] = nl;
        ncount_out[c.pix] = nc;
    }
}

template <int TW, int TH, bool HAS_N>
__global__ __launch_bounds__(TW *TH) void k_render_bwd(const ViewDesc *__restrict__ views, int V,
                                                        const uint32_t *__restrict__ ts,
                                                        const uint32_t *__restrict__ te,
                                                        const uint32_t *__restrict__ pval,
                                                        const Rec *__restrict__ rec, KParams kp, int64_t NPX,
                                                        fm_outputs out, fm_grad_outputs gout,
                                                        const uint32_t *__restrict__ nlast_in,
                                                        float *__restrict__ grad) {
    using Gm = Geo<TW, TH>;
    __shared__ Rec srec[Gm::NT];
    __shared__ uint32_t sval[Gm::NT];
    __shared__ uint32_t smax;
    const PixelCtx c = pixel_ctx<TW, TH>(views, V, ts, te);
    float g[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float S = 0.f;
    uint32_t nl = 0;
    if (c.inside) {
        const int64_t q = c.pix;
        if (gout.rgb) { g[0] = gout.rgb[q]; g[1] = gout.rgb[NPX + q]; g[2] = gout.rgb[2 * NPX + q]; }
        if (gout.depth) g[3] = gout.depth[q];
        if (HAS_N) { g[4] = gout.normal[q]; g[5] = gout.normal[NPX + q]; g[6] = gout.normal[2 * NPX + q]; }
        if (gout.alpha) g[7] = gout.alpha[q];
        bool any = false;
#pragma unroll
        for (int k = 0; k < 8; ++k) any |= g[k] != 0.f;
        if (any) {
            nl = nlast_in[q];
            S = g[0] * out.rgb[q] + g[1] * out.rgb[NPX + q] + g[2] * out.rgb[2 * NPX + q] + g[3] * out.depth[q] +
                g[7] * out.alpha[q];
            if (HAS_N) S += g[4] * out.normal[q] + g[5] * out.normal[NPX + q] + g[6] * out.normal[2 * NPX + q];
        }
    }
    const uint32_t maxlast = block_max<Gm::NT>(nl, &smax);
    if (maxlast == 0) return;
    tile_backward<TW, TH, HAS_N>(c, pval, rec, kp, srec, sval, g, S, nl, maxlast, grad);
}

template <int TW, int TH>
__global__ __launch_bounds__(TW *TH) void k_render_fused(const ViewDesc *__restrict__ views, int V,
                                                          const uint32_t *__restrict__ ts,
                                                          const uint32_t *__restrict__ te,
                                                          const uint32_t *__restrict__ pval,
                                                          const Rec *__restrict__ rec, KParams kp, int64_t NPX,
                                                          fm_outputs out, LossArgs la, float *__restrict__ tfinal,
                                                          uint32_t *__restrict__ nlast_out,
                                                          uint32_t *__restrict__ ncount_out, float *__restrict__ grad,
                                                          float *__restrict__ loss_part) {
    using Gm = Geo<TW, TH>;
    __shared__ Rec srec[Gm::NT];
    __shared__ uint32_t sval[Gm::NT];
    __shared__ uint32_t smax;
    __shared__ float sred[Gm::NW];
    const PixelCtx c = pixel_ctx<TW, TH>(views, V, ts, te);
    float acc[8], T;
    uint32_t nl, nc;
    tile_forward<TW, TH>(c, pval, rec, kp, srec, sval, acc, T, nl, nc);
    float g[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float S = 0.f, l = 0.f;
    if (c.inside) {
        const int64_t q = c.pix;
        const float o0 = acc[0] + T * kp.bg[0], o1 = acc[1] + T * kp.bg[1], o2 = acc[2] + T * kp.bg[2];
        out.rgb[q] = o0;
        out.rgb[NPX + q] = o1;
        out.rgb[2 * NPX + q] = o2;
        out.depth[q] = acc[3];
        out.normal[q] = acc[4];
        out.normal[NPX + q] = acc[5];
        out.normal[2 * NPX + q] = acc[6];
        out.alpha[q] = acc[7];
        tfinal[q] = T;
        nlast_out[q] = nl;
        ncount_out[q] = nc;
        const bool m = la.mask ? (la.mask[q] != 0) : true;
        if (m) {
            const float npx = (float)c.W * (float)c.H;
            const float k_rgb = la.w_rgb / (3.f * npx);
            const float o[3] = {o0, o1, o2};
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                const float d = o[ch] - la.target_rgb[ch * NPX + q];
                l += k_rgb * fabsf(d);
                g[ch] = d > 0.f ? k_rgb : (d < 0.f ? -k_rgb : 0.f);
            }
            if (la.w_depth != 0.f && la.target_depth) {
                const float k_d = la.w_depth / npx;
                const float d = acc[3] - la.target_depth[q];
                l += k_d * fabsf(d);
                g[3] = d > 0.f ? k_d : (d < 0.f ? -k_d : 0.f);
            }
            S = g[0] * o0 + g[1] * o1 + g[2] * o2 + g[3] * acc[3];
        } else {
            nl = 0;
        }
    } else {
        nl = 0;
    }
    const float lsum = block_sum<Gm::NT>(l, sred);
    if (threadIdx.x == 0) loss_part[blockIdx.x] = lsum;
    const uint32_t maxlast = block_max<Gm::NT>(nl, &smax);
    if (maxlast == 0) return;
    tile_backward<TW, TH, false>(c, pval, rec, kp, srec, sval, g, S, nl, maxlast, grad);
}

__global__ __launch_bounds__(1024) void k_loss_reduce(const float *__restrict__ part, int64_t n,
                                                       float *__restrict__ loss) {
    __shared__ float red[16];
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < n; i += 1024) s += part[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < 16; ++k) t += red[k];
        *loss += t;
    }
}

template <int TW, int TH>
hipError_t fwd_t(const Plan &p, void *ws, const KParams &kp, const fm_outputs &out, hipStream_t st) {
    const uint32_t *pval = at<uint32_t>(ws, p.pairs_in_alt ? p.o_pval2 : p.o_pval);
    hipLaunchKernelGGL((k_render_fwd<TW, TH>), dim3((unsigned)p.T), dim3(TW * TH), 0, st,
                       at<ViewDesc>(ws, p.o_views), p.V, at<uint32_t>(ws, p.o_tstart),
                       at<uint32_t>(ws, p.o_tend), pval, at<Rec>(ws, p.o_rec), kp, p.NPX, out,
                       at<float>(ws, p.o_tfinal), at<uint32_t>(ws, p.o_nlast), at<uint32_t>(ws, p.o_ncount));
    return hipGetLastError();
}

template <int TW, int TH>
hipError_t bwd_t(const Plan &p, void *ws, const KParams &kp, const fm_outputs &out, const fm_grad_outputs &g,
                 hipStream_t st) {
    const uint32_t *pval = at<uint32_t>(ws, p.pairs_in_alt ? p.o_pval2 : p.o_pval);
    if (g.normal)
        hipLaunchKernelGGL((k_render_bwd<TW, TH, true>), dim3((unsigned)p.T), dim3(TW * TH), 0, st,
                           at<ViewDesc>(ws, p.o_views), p.V, at<uint32_t>(ws, p.o_tstart),
                           at<uint32_t>(ws, p.o_tend), pval, at<Rec>(ws, p.o_rec), kp, p.NPX, out, g,
                           at<uint32_t>(ws, p.o_nlast), at<float>(ws, p.o_grad));
    else
        hipLaunchKernelGGL((k_render_bwd<TW, TH, false>), dim3((unsigned)p.T), dim3(TW * TH), 0, st,
                           at<ViewDesc>(ws, p.o_views), p.V, at<uint32_t>(ws, p.o_tstart),
                           at<uint32_t>(ws, p.o_tend), pval, at<Rec>(ws, p.o_rec), kp, p.NPX, out, g,
                           at<uint32_t>(ws, p.o_nlast), at<float>(ws, p.o_grad));
    return hipGetLastError();
}

template <int TW, int TH>
hipError_t fused_t(const Plan &p, void *ws, const KParams &kp, const LossArgs &la, const fm_outputs &out,
                   hipStream_t st) {
    const uint32_t *pval = at<uint32_t>(ws, p.pairs_in_alt ? p.o_pval2 : p.o_pval);
    hipLaunchKernelGGL((k_render_fused<TW, TH>), dim3((unsigned)p.T), dim3(TW * TH), 0, st,
                       at<ViewDesc>(ws, p.o_views), p.V, at<uint32_t>(ws, p.o_tstart),
                       at<uint32_t>(ws, p.o_tend), pval, at<Rec>(ws, p.o_rec), kp, p.NPX, out, la,
                       at<float>(ws, p.o_tfinal), at<uint32_t>(ws, p.o_nlast), at<uint32_t>(ws, p.o_ncount),
                       at<float>(ws, p.o_grad), at<float>(ws, p.o_loss));
    return hipGetLastError();
}

}  // namespace

bool tile_shape_supported(int tw, int th) {
    return (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 16 && th == 16) ||
           (tw == 32 && th == 8);
}

#define FM_DISPATCH(FN, ...)                                                     \
    do {                                                                         \
        if (p.tile_w == 16 && p.tile_h == 16) return FN<16, 16>(__VA_ARGS__);    \
        if (p.tile_w == 8 && p.tile_h == 8) return FN<8, 8>(__VA_ARGS__);        \
        if (p.tile_w == 16 && p.tile_h == 8) return FN<16, 8>(__VA_ARGS__);      \
        if (p.tile_w == 32 && p.tile_h == 8) return FN<32, 8>(__VA_ARGS__);      \
        return hipErrorInvalidValue;                                             \
    } while (0)

hipError_t launch_render_fwd(const Plan &p, void *ws, const KParams &kp, const fm_outputs &out,
                             hipStream_t st) {
    if (p.T == 0) return hipSuccess;
    FM_DISPATCH(fwd_t, p, ws, kp, out, st);
}

hipError_t launch_render_bwd(const Plan &p, void *ws, const KParams &kp, const fm_outputs &out,
                             const fm_grad_outputs &g, hipStream_t st) {
    if (p.T == 0) return hipSuccess;
    FM_DISPATCH(bwd_t, p, ws, kp, out, g, st);
}

hipError_t launch_render_fused(const Plan &p, void *ws, const KParams &kp, const LossArgs &la,
                               const fm_outputs &out, hipStream_t st) {
    if (p.T == 0) return hipSuccess;
    FM_DISPATCH(fused_t, p, ws, kp, la, out, st);
}

hipError_t launch_loss_reduce(const Plan &p, void *ws, float *loss, hipStream_t st) {
    if (p.T == 0 || !loss) return hipSuccess;
    hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(1024), 0, st, at<float>(ws, p.o_loss), p.T, loss);
    return hipGetLastError();
}

}  // namespace fm
