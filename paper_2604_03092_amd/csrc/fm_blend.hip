// fm_blend.hip -- per-tile front-to-back compositing (Eq. 1) and its adjoint
// on gfx950.
//
// One wave64 per tile.  The tile is a grid of 8x8 pixel blocks; lane l owns
// pixel (l mod 8, l / 8) of every block, so each lane carries one pixel
// "slot" per block (1, 2 or 4 slots).  The tile's depth-ordered surfels are
// staged through LDS 64 at a time and read as broadcasts; per surfel, the
// pair's block mask (exact support-ellipse culling) and the set of slots
// still compositing select the slots to evaluate with scalar tests.  The
// surfel's record is read once per tile, and in the adjoint the slots'
// gradients are summed in registers before one cross-lane reduction.
//
// Backward (forward order, no per-pixel lists): with f_k = g . (c_k, z_k,
// n_k, 1) and S = g . (I, D, N, A) known from the forward outputs, the
// adjoint of the compositing is
//     dL/dalpha_k = T_k f_k - (S - S_k) / (1 - alpha_k),   S_k = sum_{j<=k} f_j alpha_j T_j,
// so the backward walks the list front to back exactly like the forward,
// recomputing T, and stops at the pixel's last contributor.  Per surfel, the
// screen-space gradients of the tile are reduced with permlane swaps + DPP and
// added into the entry's gradient slot with one coalesced 16-float atomic
// group (plus one for the last normal component when normals carry a
// gradient).  With deterministic sums they are stored instead into a slot of
// the pair's own (per wave of the tile), and k_det_reduce sums each entry's
// slots in a fixed order.
//
// A 32x32 tile runs as four 16x16 quadrant waves over one shared list.
#include <algorithm>

#include "fm_internal.h"
#include "fm_wave.h"

namespace fm {

namespace {

struct Surf {
    float c00, c01, c02, c10, c11, c12, c20, c21, c22;
    float sig, r, g, b, n0, n1, n2, z, xs, ys, lsig;
};

__device__ __forceinline__ void load_surf(const Rec *rp, Surf &s) {
    const float4 *p = reinterpret_cast<const float4 *>(rp);
    const float4 a = p[0], b = p[1], c = p[2], d = p[3], e = p[4];
    s.c00 = a.x; s.c01 = a.y; s.c02 = a.z; s.c10 = a.w;
    s.c11 = b.x; s.c12 = b.y; s.c20 = b.z; s.c21 = b.w;
    s.c22 = c.x; s.sig = c.y; s.r = c.z; s.g = c.w;
    s.b = d.x; s.n0 = d.y; s.n1 = d.z; s.n2 = d.w;
    s.z = e.x; s.xs = e.y; s.ys = e.z; s.lsig = e.w;
}

// Ray-splat intersection at the pixel centre (px, py), evaluated for every
// lane without branches.  In the surfel's shifted pixel frame the ray meets
// the plane at (u, v) = (w0, w1) / w2 with w = c0 + x' c2 - y' c1.
// Stage 1 decides `in`: the lane is live and u^2 + v^2 <= rho_max^2 (a ray
// with w2^2 below 1e-30, parallel to the plane to FP32 precision, is out).
// Stage 2 evaluates sigma G = exp2(log2(sigma) - r^2 log2(e) / 2) (G =
// exp(-r^2/2), one fused multiply-add in the exponent) and alpha =
// min(alpha_max, sigma G), with `hit` = in and sigma G >= alpha_min.  Lanes that miss get alpha = 0,
// so T and the weights do not move; the adjoint zeroes their gradient terms.  Forward and backward run the same
// instructions on the same inputs and so take the same decisions.
constexpr float kMinDen = 1e-30f;

struct Hit {
    float xp, yp, w0, w1, w2, num, den, rden, r2;
    float at, alpha;
    bool in, hit;
};

__device__ __forceinline__ void splat_geom(const Surf &s, float px, float py, float rho2, bool live, Hit &h) {
#pragma clang fp contract(off)
    h.xp = px - s.xs;
    h.yp = py - s.ys;
    h.w0 = fmaf(h.xp, s.c20, fmaf(-h.yp, s.c10, s.c00));
    h.w1 = fmaf(h.xp, s.c21, fmaf(-h.yp, s.c11, s.c01));
    h.w2 = fmaf(h.xp, s.c22, fmaf(-h.yp, s.c12, s.c02));
    h.num = fmaf(h.w0, h.w0, h.w1 * h.w1);
    h.den = h.w2 * h.w2;
    h.in = live && (h.num <= rho2 * h.den) && (h.den > kMinDen);
}

// SAFE (adjoint): lanes that are not `in` get rden = 1 and r2 = 0, so their
// G, sigma G and 1/w2^2 stay finite; the forward needs only alpha and skips it.
template <bool SAFE>
__device__ __forceinline__ void splat_alpha(const Surf &s, float amin, float amax, Hit &h) {
#pragma clang fp contract(off)
    h.rden = __builtin_amdgcn_rcpf(SAFE ? (h.in ? h.den : 1.f) : h.den);
    h.r2 = SAFE ? (h.in ? h.num * h.rden : 0.f) : h.num * h.rden;
    h.at = __builtin_amdgcn_exp2f(fmaf(h.r2, -0.72134752044448170368f, s.lsig));  // sigma exp(-r2/2)
    h.hit = h.in && (h.at >= amin);
    // min(alpha_max, sigma G) on the bit patterns: both are >= 0, where the
    // IEEE order is the unsigned-integer order (and no canonicalisation is
    // needed; a NaN sigma G of a missing lane gives alpha_max, then 0)
    const uint32_t ub = __float_as_uint(h.at), um = __float_as_uint(amax);
    h.alpha = h.hit ? __uint_as_float(ub < um ? ub : um) : 0.f;
}

// Launch geometry of the blend kernels.  A tile of TW x TH pixels is a grid
// of 8x8 blocks, which its pair masks mark.  Without SPLIT one wave renders
// the whole tile as NB slots of 8x8 blocks per lane, except 32x32 tiles,
// which four 16x16 quadrant waves traverse (their pair masks mark quadrants).
// With SPLIT (16x8, 16x16 and 32x8 tiles) every 8x8 block of the tile gets a
// wave of its own, NB = 1: more, shorter waves over the same list, for
// batches too small to fill the chip.  A wave of a tile with several waves
// takes the mask bit of its block or quadrant.  DEPTH: records staged in LDS
// per batch (32, 64 or 128; 64 is one per lane).
template <int TW_, int TH_, bool SPLIT_ = false, int DEPTH_ = 64> struct Geo {
    static constexpr int TW = TW_, TH = TH_, DEPTH = DEPTH_;
    static constexpr bool BIG = TW == 32 && TH == 32;
    static constexpr bool SPLIT = SPLIT_ && !BIG && (TW > 8 || TH > 8);
    static constexpr bool QUAD = BIG || SPLIT;  // several waves per tile, one per mask bit
    static constexpr int WTW = BIG ? 16 : (SPLIT ? 8 : TW);
    static constexpr int WTH = BIG ? 16 : (SPLIT ? 8 : TH);
    static constexpr int QX = TW / WTW;
    static constexpr int NQ = QX * (TH / WTH);  // waves per tile
    static constexpr int BW = WTW / 8;
    static constexpr int BH = WTH / 8;
    static constexpr int NB = BW * BH;  // pixel slots per lane
    static_assert(DEPTH == 32 || DEPTH == 64 || DEPTH == 128, "LDS batch depth");
};

// Deterministic-gradient side of a pair list (meta == nullptr otherwise):
// meta[emission index] = the pair's value, cap = pair capacity, part = the
// partial gradient slots, one per (emission index, wave of the tile), and
// flag = one byte per slot, set when the wave has written the slot (slots
// whose flag is clear are read as zero).
struct PairMeta {
    const uint32_t *meta;
    uint32_t cap;
    float *part;
    uint8_t *flag;
};

struct TileCtx {
    int view, W, H;
    int64_t pix_base;      // first pixel of the view in the output planes
    uint32_t start, end;   // the tile's range in the sorted pair list
    uint32_t n_entries;
    int tile;  // batch-global tile id
    int quad;  // the wave's block or quadrant of a tile with several waves (0 otherwise)
};

template <class G> struct Slots {
    float px[G::NB], py[G::NB];
    int64_t pix[G::NB];
    bool inside[G::NB];
};

template <class G>
__device__ __forceinline__ TileCtx tile_ctx(const ViewDesc *views, int V, const uint32_t *ts,
                                            const uint32_t *te, const uint32_t *order, Slots<G> &sl) {
    using Gm = G;
    constexpr int TW = G::TW, TH = G::TH;
    TileCtx c;
    // runs of 16 consecutive blocks share an L2 (the quadrants of a tile
    // are consecutive blocks)
    const int lb = (int)xcd_chunked<16>(blockIdx.x, gridDim.x);
    const int rank = lb / Gm::NQ;
    c.quad = lb - rank * Gm::NQ;
    const int tile = order ? (int)order[rank] : rank;  // longest list first, or image order
    c.tile = tile;
    c.view = view_of_tile(views, V, tile);
    const ViewDesc &vd = views[c.view];
    const int local = tile - vd.tile_base;
    const int tx = local % vd.tiles_x, ty = local / vd.tiles_x;
    c.W = vd.width;
    c.H = vd.height;
    c.pix_base = vd.pixel_offset;
    c.start = ts[tile];
    c.end = te[tile];
    if (c.start > c.end) c.start = c.end;  // a tile without pairs
    c.n_entries = (uint32_t)views[V - 1].entry_base + (((uint32_t)views[V - 1].n + 255u) & ~255u);
    const int lane = threadIdx.x;
#pragma unroll
    for (int q = 0; q < Gm::NB; ++q) {
        const int col = tx * TW + (c.quad % Gm::QX) * Gm::WTW + 8 * (q % Gm::BW) + (lane & 7);
        const int row = ty * TH + (c.quad / Gm::QX) * Gm::WTH + 8 * (q / Gm::BW) + (lane >> 3);
        sl.inside[q] = col < c.W && row < c.H;
        sl.pix[q] = c.pix_base + (int64_t)row * c.W + col;
        sl.px[q] = (float)col + 0.5f;
        sl.py[q] = (float)row + 0.5f;
    }
    return c;
}

// Stage up to G::DEPTH pairs of the tile list into LDS (one per lane and
// 64-pair half).  Entries out of range (impossible for emitted pairs) get an
// empty block mask.  In a wave of a tile with several waves (QUAD) the
// pair's bit of the wave's block or quadrant becomes a mask of all slots.
// Deterministic lists (meta non-null) hold emission indices: the index goes
// to sj and meta gives the pair's value.
template <class G>
__device__ __forceinline__ int stage(const TileCtx &c, uint32_t base, uint32_t end,
                                     const uint32_t *__restrict__ pval, const Rec *__restrict__ rec,
                                     Rec *srec, uint32_t *sval, const PairMeta &pm, uint32_t *sj) {
    const int cntb = (int)min((uint32_t)G::DEPTH, end - base);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < (G::DEPTH + 63) / 64; ++h) {
        const int i = h * 64 + (int)threadIdx.x;
        if (i < cntb) {
            uint32_t pv = pval[base + i];
            if (pm.meta) {
                sj[i] = pv;
                pv = pv < pm.cap ? pm.meta[pv] : 0u;  // (an index past the capacity cannot occur)
            }
            const bool ok = (pv & kEntryMask) < c.n_entries;
            if (G::QUAD)
                pv = (pv & kEntryMask) | (((pv >> (kMaskShift + c.quad)) & 1u) ? (0xFu << kMaskShift) : 0u);
            sval[i] = ok ? pv : 0u;
            if (ok) srec[i] = rec[pv & kEntryMask];
        }
    }
    __syncthreads();
    return cntb;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, off);
        v = o > v ? o : v;
    }
    return v;
}

// Forward traversal of the tile list for every slot of the lane.
// acc = (r, g, b, depth, nx, ny, nz, A) per slot; slast[q] (wave-uniform) is
// one past the last list position where a pixel of the slot was inside a
// surfel's support, a bound on its last contributor for the adjoint.  A
// pixel that is outside the image or has stopped compositing carries x =
// NaN, which fails every support test; slots whose pixels have all stopped
// are dropped from the live set every 8 list positions.  COUNT: also count
// each pixel's contributors (ncount; the fused path skips it).
template <class G, bool COUNT>
__device__ __forceinline__ void tile_forward(const TileCtx &c, const Slots<G> &sl,
                                             const uint32_t *__restrict__ pval, const Rec *__restrict__ rec,
                                             const KParams &kp, Rec *srec, uint32_t *sval,
                                             const PairMeta &pm, uint32_t *sj,
                                             float (&acc)[G::NB][8], float (&T)[G::NB],
                                             uint32_t (&slast)[G::NB],
                                             uint32_t (&ncount)[G::NB]) {
#pragma clang fp contract(off)
    using Gm = G;
    const float rho2 = kp.rho_max * kp.rho_max;
    const float amax = kp.alpha_max;
    const float nan = __builtin_nanf("");
    float px[Gm::NB];
    uint32_t live = 0;
#pragma unroll
    for (int q = 0; q < Gm::NB; ++q) {
        px[q] = sl.inside[q] ? sl.px[q] : nan;
        T[q] = 1.f;
        slast[q] = 0;
        ncount[q] = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[q][k] = 0.f;
        if (ballot64(sl.inside[q]) != 0) live |= 1u << q;
    }
    for (uint32_t base = c.start; base < c.end && live != 0; base += G::DEPTH) {
        const int cntb = stage<Gm>(c, base, c.end, pval, rec, srec, sval, pm, sj);
        for (int j = 0; j < cntb; ++j) {
            const uint32_t m = (__builtin_amdgcn_readfirstlane(sval[j]) >> kMaskShift) & live;
            if (m != 0) {
                Surf s;
                load_surf(&srec[j], s);
#pragma unroll
                for (int q = 0; q < Gm::NB; ++q) {
                    if (((m >> q) & 1u) == 0) continue;
                    Hit h;
                    splat_geom(s, px[q], sl.py[q], rho2, true, h);
                    if (ballot64(h.in) == 0) continue;
                    slast[q] = base - c.start + (uint32_t)j + 1u;
                    splat_alpha<false>(s, kp.alpha_min, amax, h);
                    const float test = T[q] * (1.f - h.alpha);
                    const bool con = h.hit && test >= kp.t_min;  // test is finite
                    const bool stop = h.hit != con;
                    const float wgt = (con ? h.alpha : 0.f) * T[q];
                    acc[q][0] = fmaf(s.r, wgt, acc[q][0]);
                    acc[q][1] = fmaf(s.g, wgt, acc[q][1]);
                    acc[q][2] = fmaf(s.b, wgt, acc[q][2]);
                    acc[q][3] = fmaf(s.z, wgt, acc[q][3]);
                    acc[q][4] = fmaf(s.n0, wgt, acc[q][4]);
                    acc[q][5] = fmaf(s.n1, wgt, acc[q][5]);
                    acc[q][6] = fmaf(s.n2, wgt, acc[q][6]);
                    acc[q][7] = acc[q][7] + wgt;
                    T[q] = con ? test : T[q];
                    if (COUNT) ncount[q] += con ? 1u : 0u;
                    px[q] = stop ? nan : px[q];
                }
            }
            if ((j & 7) == 7) {
#pragma unroll
                for (int q = 0; q < Gm::NB; ++q)
                    if (ballot64(px[q] == px[q]) == 0) live &= ~(1u << q);
                if (live == 0) break;
            }
        }
    }
}

// Adjoint terms of one hit slot, added into the lane's per-surfel gradient
// registers (gr: dL/dc0[3], dL/dc1[3], dL/dc2[3], sigma dL/dsigma, dL/d(r, g, b),
// dL/dz, dL/dn[0..1]; gn2: dL/dn[2]).  FIRST: the first slot of the surfel,
// which assigns instead of adding.  Also steps S_k and T of the slot.
template <bool FIRST, bool HAS_N>
__device__ __forceinline__ void adjoint_terms(const Hit &h, const Surf &s, const float (&gq)[8], float Sq,
                                              float &Skq, float &Tq, float amax, float (&gr)[16], float &gn2) {
#pragma clang fp contract(off)
    auto mac = [](float &d, float a, float b) { d = FIRST ? a * b : fmaf(a, b, d); };
    auto add = [](float &d, float v) { d = FIRST ? v : d + v; };
    // lanes that miss have alpha = 0: wgt = 0 and T is unchanged
    const float test = Tq * (1.f - h.alpha);
    const float wgt = h.alpha * Tq;
    float f = fmaf(gq[0], s.r, fmaf(gq[1], s.g, fmaf(gq[2], s.b, fmaf(gq[3], s.z, gq[7]))));
    if (HAS_N) f = fmaf(gq[4], s.n0, fmaf(gq[5], s.n1, fmaf(gq[6], s.n2, f)));
    Skq = fmaf(f, wgt, Skq);
    const float dal = fmaf(-(Sq - Skq), __builtin_amdgcn_rcpf(1.f - h.alpha), Tq * f);
    // alpha = sigma G below the clamp; above it alpha carries no gradient
    const float du = (h.hit && h.at <= amax) ? dal : 0.f;
    mac(gr[10], gq[0], wgt);
    mac(gr[11], gq[1], wgt);
    mac(gr[12], gq[2], wgt);
    mac(gr[13], gq[3], wgt);
    if (HAS_N) {
        mac(gr[14], gq[4], wgt);
        mac(gr[15], gq[5], wgt);
        mac(gn2, gq[6], wgt);
    }
    // G = exp(-r2/2), r2 = (w0^2 + w1^2) / w2^2, w = c0 + x' c2 - y' c1:
    // sigma dL/dsigma = du sigma G (divided by sigma after the tile's
    // reduction), dL/dr2 = -du sigma G / 2, and
    // dr2/dw = (2 w0, 2 w1, -2 r2 w2) / w2^2
    const float dua = du * h.at;
    add(gr[9], dua);
    // (a lane that misses has du = 0 and finite rden, r2 and w -- the
    // projection culls records with coefficients beyond 1e30 -- so its terms
    // are signed zeros)
    const float kk = -dua * h.rden;
    const float gw0 = kk * h.w0, gw1 = kk * h.w1, gw2 = -(kk * h.r2) * h.w2;
    add(gr[0], gw0);
    add(gr[1], gw1);
    add(gr[2], gw2);
    mac(gr[3], -h.yp, gw0);
    mac(gr[4], -h.yp, gw1);
    mac(gr[5], -h.yp, gw2);
    mac(gr[6], h.xp, gw0);
    mac(gr[7], h.xp, gw1);
    mac(gr[8], h.xp, gw2);
    Tq = test;
}

// Adjoint traversal.  g[q] = dL/d(r, g, b, depth, nx, ny, nz, A) of slot q's
// pixel, S[q] = g[q] . outputs, Tf[q] = its final transmittance (1 for a
// pixel without gradient), bound[q] = the slot's traversal bound (any value
// >= one past its last contributor).  Every contribution lowers T strictly
// (alpha >= alpha_min >= 1e-6 and T >= t_min stays normal), and the
// recomputed T repeats the forward's exactly, so a pixel still has
// contributions ahead exactly while T > Tf.  HAS_N: the normal map carries a
// gradient.
template <class G, bool HAS_N, bool DET>
__device__ __forceinline__ void tile_backward(const TileCtx &c, const Slots<G> &sl,
                                              const uint32_t *__restrict__ pval, const Rec *__restrict__ rec,
                                              const KParams &kp, Rec *srec, uint32_t *sval,
                                              const PairMeta &pm, uint32_t *sj,
                                              const float (&g)[G::NB][8], const float (&S)[G::NB],
                                              const float (&Tf)[G::NB],
                                              const uint32_t (&bound)[G::NB], float *__restrict__ grad) {
    using Gm = G;
    const float rho2 = kp.rho_max * kp.rho_max;
    const float amax = kp.alpha_max;
    float T[Gm::NB], Sk[Gm::NB];
    uint32_t smax[Gm::NB];
    uint32_t maxlast = 0;
#pragma unroll
    for (int q = 0; q < Gm::NB; ++q) {
        T[q] = 1.f;
        Sk[q] = 0.f;
        smax[q] = bound[q];
        maxlast = smax[q] > maxlast ? smax[q] : maxlast;
    }
    const uint32_t len = c.end - c.start;
    const uint32_t end = c.start + (maxlast < len ? maxlast : len);
    const int comp = wave_reduce16_component();
    for (uint32_t base = c.start; base < end; base += G::DEPTH) {
        const int cntb = stage<Gm>(c, base, end, pval, rec, srec, sval, pm, sj);
        const uint32_t kbase = base - c.start;
        for (int j = 0; j < cntb; ++j) {
            const uint32_t k = kbase + (uint32_t)j;
            uint32_t m = __builtin_amdgcn_readfirstlane(sval[j]) >> kMaskShift;
#pragma unroll
            for (int q = 0; q < Gm::NB; ++q)
                if (k >= smax[q]) m &= ~(1u << q);
            if (m == 0) continue;
            Surf s;
            load_surf(&srec[j], s);
            // per-surfel gradient registers, written (not added) by the first hit
            // slot, so nothing is carried from the previous surfel; without
            // normal gradients gr[14], gr[15] are zero
            float gr[16], gn2;
            if (!HAS_N) gr[14] = gr[15] = 0.f;
            bool first = true;
#pragma unroll
            for (int q = 0; q < Gm::NB; ++q) {
                if (((m >> q) & 1u) == 0) continue;
                Hit h;
                splat_geom(s, sl.px[q], sl.py[q], rho2, T[q] > Tf[q], h);
                if (ballot64(h.in) == 0) continue;
                splat_alpha<true>(s, kp.alpha_min, amax, h);
                // no early-out when no lane is hit (rare once a lane is inside):
                // a missing lane's terms are exact zeros
                if (first)
                    adjoint_terms<true, HAS_N>(h, s, g[q], S[q], Sk[q], T[q], amax, gr, gn2);
                else
                    adjoint_terms<false, HAS_N>(h, s, g[q], S[q], Sk[q], T[q], amax, gr, gn2);
                first = false;
            }
            if (first) continue;  // no lane of the tile is hit by this surfel
            float r = wave_reduce16(gr);
            if (comp == 9) r *= __builtin_amdgcn_rcpf(s.sig);  // sigma dL/dsigma -> dL/dsigma
            if (DET) {  // this wave's own partial slot of the pair, every float of it, then its flag
                const int64_t slot = (int64_t)sj[j] * Gm::NQ + c.quad;
                float *dst = pm.part + slot * kp.gstride;
                if (comp >= 0) dst[comp] = r;  // without normal gradients 14 and 15 hold zeros
                if (HAS_N) {
                    const float t2 = wave_sum(gn2);
                    if (lane_id() == 0) {
                        dst[16] = t2;
                        dst[17] = dst[18] = dst[19] = 0.f;
                    }
                }
                if (lane_id() == 0) pm.flag[slot] = 1;
            } else {
                float *dst = grad + (int64_t)(sval[j] & kEntryMask) * kp.gstride;
                if (comp >= 0 && (HAS_N || comp < 14)) atomicAdd(dst + comp, r);  // 14, 15: normal terms
                if (HAS_N) {
                    const float t2 = wave_sum(gn2);
                    if (lane_id() == 0) atomicAdd(dst + 16, t2);
                }
            }
        }
    }
}

// Map-fusion pruning score traversal (forward side, no adjoint): walks the
// tile list again like the forward, recomputing T exactly, for the slots
// whose pixel is flagged (flag[q], with final transmittance Tf[q]); every
// surfel's weights alpha T on the flagged pixels of the wave are summed and
// added into the first float of its entry's gradient slot (one atomic per
// (tile, surfel) that touches a flagged pixel).
template <class G>
__device__ __forceinline__ void tile_score(const TileCtx &c, const Slots<G> &sl,
                                           const uint32_t *__restrict__ pval, const Rec *__restrict__ rec,
                                           const KParams &kp, Rec *srec, uint32_t *sval, const PairMeta &pm,
                                           uint32_t *sj, const bool (&flag)[G::NB],
                                           const float (&Tf)[G::NB],
                                           const uint32_t (&bound)[G::NB], float *__restrict__ grad) {
#pragma clang fp contract(off)
    using Gm = G;
    const float rho2 = kp.rho_max * kp.rho_max;
    float T[Gm::NB];
    uint32_t smax[Gm::NB];
    uint32_t maxlast = 0;
#pragma unroll
    for (int q = 0; q < Gm::NB; ++q) {
        T[q] = 1.f;
        // a slot without flagged pixels is not traversed
        smax[q] = ballot64(flag[q]) != 0 ? bound[q] : 0u;
        maxlast = smax[q] > maxlast ? smax[q] : maxlast;
    }
    const uint32_t len = c.end - c.start;
    const uint32_t end = c.start + (maxlast < len ? maxlast : len);
    for (uint32_t base = c.start; base < end; base += G::DEPTH) {
        const int cntb = stage<Gm>(c, base, end, pval, rec, srec, sval, pm, sj);
        const uint32_t kbase = base - c.start;
        for (int j = 0; j < cntb; ++j) {
            const uint32_t k = kbase + (uint32_t)j;
            uint32_t m = __builtin_amdgcn_readfirstlane(sval[j]) >> kMaskShift;
#pragma unroll
            for (int q = 0; q < Gm::NB; ++q)
                if (k >= smax[q]) m &= ~(1u << q);
            if (m == 0) continue;
            Surf s;
            load_surf(&srec[j], s);
            float w = 0.f;
            bool any = false;
#pragma unroll
            for (int q = 0; q < Gm::NB; ++q) {
                if (((m >> q) & 1u) == 0) continue;
                Hit h;
                splat_geom(s, sl.px[q], sl.py[q], rho2, flag[q] && T[q] > Tf[q], h);
                if (ballot64(h.in) == 0) continue;
                splat_alpha<false>(s, kp.alpha_min, kp.alpha_max, h);
                // alpha = 0 where the surfel misses: T and the sum do not move
                w = fmaf(h.alpha, T[q], w);
                T[q] = T[q] * (1.f - h.alpha);
                any = true;
            }
            if (!any) continue;
            const float tot = wave_sum(w);
            // (staging has mapped a deterministic list's emission index to the pair value)
            if (lane_id() == 0 && tot != 0.f) atomicAdd(grad + (int64_t)(sval[j] & kEntryMask) * kp.gstride, tot);
        }
    }
}

// ---------------------------------------------------------------------------
template <class G>
__global__ __launch_bounds__(64) void k_render_fwd(const ViewDesc *__restrict__ views, int V,
                                                    const uint32_t *__restrict__ ts, const uint32_t *__restrict__ te,
                                                    const uint32_t *__restrict__ order,
                                                    const uint32_t *__restrict__ pval, const Rec *__restrict__ rec,
                                                    KParams kp, int64_t NPX, fm_outputs out,
                                                    float *__restrict__ tfinal, uint32_t *__restrict__ nlast_out,
                                                    uint32_t *__restrict__ ncount_out, PairMeta pm) {
    using Gm = G;
    __shared__ Rec srec[G::DEPTH];
    __shared__ uint32_t sval[G::DEPTH], sj[G::DEPTH];
    Slots<G> sl;
    const TileCtx c = tile_ctx<G>(views, V, ts, te, order, sl);
    float acc[Gm::NB][8], T[Gm::NB];
    uint32_t slast[Gm::NB], nc[Gm::NB];
    tile_forward<G, true>(c, sl, pval, rec, kp, srec, sval, pm, sj, acc, T, slast, nc);
#pragma unroll
    for (int q = 0; q < Gm::NB; ++q) {
        if (!sl.inside[q]) continue;
        const int64_t p = sl.pix[q];
        out.rgb[p] = acc[q][0] + T[q] * kp.bg[0];
        out.rgb[NPX + p] = acc[q][1] + T[q] * kp.bg[1];
        out.rgb[2 * NPX + p] = acc[q][2] + T[q] * kp.bg[2];
        out.depth[p] = acc[q][3];
        out.normal[p] = acc[q][4];
        out.normal[NPX + p] = acc[q][5];
        out.normal[2 * NPX + p] = acc[q][6];
        out.alpha[p] = acc[q][7];
        tfinal[p] = T[q];
        nlast_out[p] = slast[q];
        ncount_out[p] = nc[q];
    }
}

template <class G, bool HAS_N, bool DET>
__global__ __launch_bounds__(64) void k_render_bwd(const ViewDesc *__restrict__ views, int V,
                                                    const uint32_t *__restrict__ ts, const uint32_t *__restrict__ te,
                                                    const uint32_t *__restrict__ order,
                                                    const uint32_t *__restrict__ pval, const Rec *__restrict__ rec,
                                                    KParams kp, int64_t NPX, fm_outputs out, fm_grad_outputs gout,
                                                    const float *__restrict__ tfinal,
                                                    const uint32_t *__restrict__ nlast_in, float *__restrict__ grad,
                                                    PairMeta pm) {
    using Gm = G;
    __shared__ Rec srec[G::DEPTH];
    __shared__ uint32_t sval[G::DEPTH], sj[G::DEPTH];
    Slots<G> sl;
    const TileCtx c = tile_ctx<G>(views, V, ts, te, order, sl);
    float g[Gm::NB][8], S[Gm::NB], Tf[Gm::NB];
    uint32_t bound[Gm::NB];
#pragma unroll
    for (int q = 0; q < Gm::NB; ++q) {
#pragma unroll
        for (int k = 0; k < 8; ++k) g[q][k] = -0.f;
        S[q] = 0.f;
        Tf[q] = 1.f;
        const uint32_t nl = sl.inside[q] ? nlast_in[sl.pix[q]] : 0u;
        bound[q] = __builtin_amdgcn_readfirstlane(wave_max_u32(nl));
        if (!sl.inside[q]) continue;
        const int64_t p = sl.pix[q];
        if (gout.rgb) { g[q][0] = gout.rgb[p]; g[q][1] = gout.rgb[NPX + p]; g[q][2] = gout.rgb[2 * NPX + p]; }
        if (gout.depth) g[q][3] = gout.depth[p];
        if (HAS_N) { g[q][4] = gout.normal[p]; g[q][5] = gout.normal[NPX + p]; g[q][6] = gout.normal[2 * NPX + p]; }
        if (gout.alpha) g[q][7] = gout.alpha[p];
        bool any = false;
#pragma unroll
        for (int k = 0; k < 8; ++k) any |= g[q][k] != 0.f;
        if (any) {
            Tf[q] = tfinal[p];
            S[q] = g[q][0] * out.rgb[p] + g[q][1] * out.rgb[NPX + p] + g[q][2] * out.rgb[2 * NPX + p] +
                   g[q][3] * out.depth[p] + g[q][7] * out.alpha[p];
            if (HAS_N)
                S[q] += g[q][4] * out.normal[p] + g[q][5] * out.normal[NPX + p] + g[q][6] * out.normal[2 * NPX + p];
        }
    }
    tile_backward<G, HAS_N, DET>(c, sl, pval, rec, kp, srec, sval, pm, sj, g, S, Tf, bound, grad);
}

template <class G, bool DET>
__global__ __launch_bounds__(64) void k_render_fused(const ViewDesc *__restrict__ views, int V,
                                                      const uint32_t *__restrict__ ts, const uint32_t *__restrict__ te,
                                                    const uint32_t *__restrict__ order,
                                                      const uint32_t *__restrict__ pval, const Rec *__restrict__ rec,
                                                      KParams kp, int64_t NPX, fm_outputs out, LossArgs la,
                                                      float *__restrict__ tfinal, uint32_t *__restrict__ nlast_out,
                                                      float *__restrict__ grad, float *__restrict__ loss_part,
                                                      PairMeta pm) {
    using Gm = G;
    __shared__ Rec srec[G::DEPTH];
    __shared__ uint32_t sval[G::DEPTH], sj[G::DEPTH];
    Slots<G> sl;
    const TileCtx c = tile_ctx<G>(views, V, ts, te, order, sl);
    float acc[Gm::NB][8], T[Gm::NB];
    uint32_t slast[Gm::NB], nc[Gm::NB];
    tile_forward<G, false>(c, sl, pval, rec, kp, srec, sval, pm, sj, acc, T, slast, nc);
    float g[Gm::NB][8], S[Gm::NB], Tf[Gm::NB];
    float l = 0.f;
    const float npx = (float)c.W * (float)c.H;
    const float k_rgb = la.w_rgb / (3.f * npx);
    const float k_d = la.w_depth / npx;
#pragma unroll
    for (int q = 0; q < Gm::NB; ++q) {
#pragma unroll
        for (int k = 0; k < 8; ++k) g[q][k] = -0.f;
        S[q] = 0.f;
        Tf[q] = 1.f;
        if (!sl.inside[q]) continue;
        const int64_t p = sl.pix[q];
        const float o0 = acc[q][0] + T[q] * kp.bg[0], o1 = acc[q][1] + T[q] * kp.bg[1],
                    o2 = acc[q][2] + T[q] * kp.bg[2];
        out.rgb[p] = o0;
        out.rgb[NPX + p] = o1;
        out.rgb[2 * NPX + p] = o2;
        out.depth[p] = acc[q][3];
        out.normal[p] = acc[q][4];
        out.normal[NPX + p] = acc[q][5];
        out.normal[2 * NPX + p] = acc[q][6];
        out.alpha[p] = acc[q][7];
        tfinal[p] = T[q];
        nlast_out[p] = slast[q];
        const bool m = la.mask ? (la.mask[p] != 0) : true;
        if (!m) continue;
        Tf[q] = T[q];
        const float o[3] = {o0, o1, o2};
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float d = o[ch] - la.target_rgb[ch * NPX + p];
            l += k_rgb * fabsf(d);
            g[q][ch] = d > 0.f ? k_rgb : (d < 0.f ? -k_rgb : 0.f);
        }
        if (la.w_depth != 0.f && la.target_depth) {
            const float d = acc[q][3] - la.target_depth[p];
            l += k_d * fabsf(d);
            g[q][3] = d > 0.f ? k_d : (d < 0.f ? -k_d : 0.f);
        }
        S[q] = g[q][0] * o0 + g[q][1] * o1 + g[q][2] * o2 + g[q][3] * acc[q][3];
    }
    const float lsum = wave_sum(l);
    // partials by (tile, wave), so the reduction's order does not depend on the schedule
    if (threadIdx.x == 0) loss_part[(int64_t)c.tile * G::NQ + c.quad] = lsum;
    tile_backward<G, false, DET>(c, sl, pval, rec, kp, srec, sval, pm, sj, g, S, Tf, slast, grad);
}

// Pruning products of map fusion: forward render (outputs written as by the
// plain forward), the per-pixel error flag (a caller mask, or mean over the
// channels of |I - I*| above tau_rgb, or |D - D*| above tau_depth with a
// depth target), then the score traversal of the same list.
template <class G>
__global__ __launch_bounds__(64) void k_render_prune(const ViewDesc *__restrict__ views, int V,
                                                      const uint32_t *__restrict__ ts, const uint32_t *__restrict__ te,
                                                      const uint32_t *__restrict__ order,
                                                      const uint32_t *__restrict__ pval, const Rec *__restrict__ rec,
                                                      KParams kp, int64_t NPX, fm_outputs out, PruneArgs pa,
                                                      float *__restrict__ tfinal, float *__restrict__ grad,
                                                      PairMeta pm) {
#pragma clang fp contract(off)
    using Gm = G;
    __shared__ Rec srec[G::DEPTH];
    __shared__ uint32_t sval[G::DEPTH], sj[G::DEPTH];
    Slots<G> sl;
    const TileCtx c = tile_ctx<G>(views, V, ts, te, order, sl);
    float acc[Gm::NB][8], T[Gm::NB];
    uint32_t slast[Gm::NB], nc[Gm::NB];
    tile_forward<G, false>(c, sl, pval, rec, kp, srec, sval, pm, sj, acc, T, slast, nc);
    bool flag[Gm::NB];
#pragma unroll
    for (int q = 0; q < Gm::NB; ++q) {
        flag[q] = false;
        if (!sl.inside[q]) continue;
        const int64_t p = sl.pix[q];
        const float o0 = acc[q][0] + T[q] * kp.bg[0], o1 = acc[q][1] + T[q] * kp.bg[1],
                    o2 = acc[q][2] + T[q] * kp.bg[2];
        out.rgb[p] = o0;
        out.rgb[NPX + p] = o1;
        out.rgb[2 * NPX + p] = o2;
        out.depth[p] = acc[q][3];
        out.normal[p] = acc[q][4];
        out.normal[NPX + p] = acc[q][5];
        out.normal[2 * NPX + p] = acc[q][6];
        out.alpha[p] = acc[q][7];
        tfinal[p] = T[q];
        bool f;
        if (pa.mask_in) {
            f = pa.mask_in[p] != 0;
        } else {
            const float e = (fabsf(o0 - pa.target_rgb[p]) + fabsf(o1 - pa.target_rgb[NPX + p])) +
                            fabsf(o2 - pa.target_rgb[2 * NPX + p]);
            f = e / 3.f > pa.tau_rgb;
            if (pa.target_depth) f = f || fabsf(acc[q][3] - pa.target_depth[p]) > pa.tau_depth;
        }
        if (pa.mask_out) pa.mask_out[p] = f ? 1 : 0;
        flag[q] = f;
    }
    tile_score<G>(c, sl, pval, rec, kp, srec, sval, pm, sj, flag, T, slast, grad);
}

__global__ __launch_bounds__(1024) void k_loss_reduce(const float *__restrict__ part, int64_t n,
                                                       float *__restrict__ loss, int overwrite) {
    __shared__ float red[16];
    // a thread sums its partials in index order; eight loads are issued
    // before they are added
    float s = 0.f;
    int64_t i = threadIdx.x;
    for (; i + 7 * 1024 < n; i += 8 * 1024) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[i + u * 1024];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; i < n; i += 1024) s += part[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int k = 0; k < 16; ++k) t += red[k];
        *loss = overwrite ? t : *loss + t;
    }
}

// The blend's tile order: a permutation written by the binning, or none
// (image order).
const uint32_t *tile_order(const Plan &p, void *ws) { return p.lpt ? at<uint32_t>(ws, p.o_torder) : nullptr; }

PairMeta pair_meta(const Plan &p, void *ws) {
    PairMeta pm;
    pm.meta = p.det ? at<uint32_t>(ws, p.o_meta) : nullptr;
    pm.cap = (uint32_t)p.cap;
    pm.part = p.det ? at<float>(ws, p.o_part) : nullptr;
    pm.flag = p.det ? at<uint8_t>(ws, p.o_pflag) : nullptr;
    return pm;
}

template <class G>
hipError_t fwd_t(const Plan &p, void *ws, const KParams &kp, const fm_outputs &out, hipStream_t st) {
    const uint32_t *pval = at<uint32_t>(ws, p.pairs_in_alt ? p.o_pval2 : p.o_pval);
    hipLaunchKernelGGL((k_render_fwd<G>), dim3((unsigned)(p.T * G::NQ)), dim3(64), 0, st,
                       at<ViewDesc>(ws, p.o_views), p.V, at<uint32_t>(ws, p.o_tstart),
                       at<uint32_t>(ws, p.o_tend), tile_order(p, ws), pval, at<Rec>(ws, p.o_rec), kp, p.NPX, out,
                       at<float>(ws, p.o_tfinal), at<uint32_t>(ws, p.o_nlast), at<uint32_t>(ws, p.o_ncount),
                       pair_meta(p, ws));
    return hipGetLastError();
}

template <class G, bool HAS_N, bool DET>
void bwd_launch(const Plan &p, void *ws, const KParams &kp, const fm_outputs &out, const fm_grad_outputs &g,
                hipStream_t st) {
    const uint32_t *pval = at<uint32_t>(ws, p.pairs_in_alt ? p.o_pval2 : p.o_pval);
    hipLaunchKernelGGL((k_render_bwd<G, HAS_N, DET>), dim3((unsigned)(p.T * G::NQ)), dim3(64), 0,
                       st, at<ViewDesc>(ws, p.o_views), p.V, at<uint32_t>(ws, p.o_tstart),
                       at<uint32_t>(ws, p.o_tend), tile_order(p, ws), pval, at<Rec>(ws, p.o_rec), kp, p.NPX, out, g,
                       at<float>(ws, p.o_tfinal), at<uint32_t>(ws, p.o_nlast), at<float>(ws, p.o_grad),
                       pair_meta(p, ws));
}

template <class G>
hipError_t bwd_t(const Plan &p, void *ws, const KParams &kp, const fm_outputs &out, const fm_grad_outputs &g,
                 hipStream_t st) {
    if (g.normal) {
        if (p.det) bwd_launch<G, true, true>(p, ws, kp, out, g, st);
        else bwd_launch<G, true, false>(p, ws, kp, out, g, st);
    } else {
        if (p.det) bwd_launch<G, false, true>(p, ws, kp, out, g, st);
        else bwd_launch<G, false, false>(p, ws, kp, out, g, st);
    }
    return hipGetLastError();
}

template <class G, bool DET>
void fused_launch(const Plan &p, void *ws, const KParams &kp, const LossArgs &la, const fm_outputs &out,
                  hipStream_t st) {
    const uint32_t *pval = at<uint32_t>(ws, p.pairs_in_alt ? p.o_pval2 : p.o_pval);
    hipLaunchKernelGGL((k_render_fused<G, DET>), dim3((unsigned)(p.T * G::NQ)), dim3(64), 0, st,
                       at<ViewDesc>(ws, p.o_views), p.V, at<uint32_t>(ws, p.o_tstart),
                       at<uint32_t>(ws, p.o_tend), tile_order(p, ws), pval, at<Rec>(ws, p.o_rec), kp, p.NPX, out, la,
                       at<float>(ws, p.o_tfinal), at<uint32_t>(ws, p.o_nlast), at<float>(ws, p.o_grad),
                       at<float>(ws, p.o_loss), pair_meta(p, ws));
}

// Deterministic sums run with the default LDS depth only (the plan forces it).
template <class G>
hipError_t fused_t(const Plan &p, void *ws, const KParams &kp, const LossArgs &la, const fm_outputs &out,
                   hipStream_t st) {
    if constexpr (G::DEPTH == 64) {
        if (p.det) {
            fused_launch<G, true>(p, ws, kp, la, out, st);
            return hipGetLastError();
        }
    }
    if (p.det) return hipErrorInvalidValue;
    fused_launch<G, false>(p, ws, kp, la, out, st);
    return hipGetLastError();
}

template <class G>
hipError_t prune_t(const Plan &p, void *ws, const KParams &kp, const PruneArgs &pa, const fm_outputs &out,
                   hipStream_t st) {
    const uint32_t *pval = at<uint32_t>(ws, p.pairs_in_alt ? p.o_pval2 : p.o_pval);
    hipLaunchKernelGGL((k_render_prune<G>), dim3((unsigned)(p.T * G::NQ)), dim3(64), 0, st,
                       at<ViewDesc>(ws, p.o_views), p.V, at<uint32_t>(ws, p.o_tstart), at<uint32_t>(ws, p.o_tend),
                       tile_order(p, ws), pval, at<Rec>(ws, p.o_rec), kp, p.NPX, out, pa,
                       at<float>(ws, p.o_tfinal), at<float>(ws, p.o_grad), pair_meta(p, ws));
    return hipGetLastError();
}

// Deterministic gradients, step 1: clear the slot flags of the stored pairs
// (n_pairs emission indices x nq waves, one byte each, four per word), since
// an adjoint writes only the slots of pairs that hit one of its pixels.
__global__ __launch_bounds__(256) void k_det_clear(uint32_t *__restrict__ flag4, const Status *st, int nq) {
    const int64_t n = ((int64_t)st->n_pairs * nq + 3) / 4;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) flag4[i] = 0u;
}

__device__ __forceinline__ void add4(float4 &a, const float4 &v) {
    a.x += v.x; a.y += v.y; a.z += v.z; a.w += v.w;
}

// Step 2: four lanes per entry in depth order, one float4 of the slot each
// (lane 0 also takes the fifth float4 of 20-float slots): the entry's pairs
// are the emission indices [off32[r], off32[r + 1]) (the last entry's run
// ends at n_pairs), so its partials are one contiguous block; the flagged
// ones are summed in index order, then wave order, and stored into the
// entry's gradient slot.
__global__ __launch_bounds__(256) void k_det_reduce(const uint32_t *__restrict__ sorted_entry,
                                                     const uint32_t *__restrict__ off32, const Status *st,
                                                     const float4 *__restrict__ part,
                                                     const uint8_t *__restrict__ flag, int nq, int gs4,
                                                     float4 *__restrict__ grad) {
    const uint32_t nv = st->n_vis, np = st->n_pairs;
    const int c4 = threadIdx.x & 3;
    const bool fifth = gs4 == 5 && c4 == 0;
    for (int64_t r = (int64_t)blockIdx.x * 64 + (threadIdx.x >> 2); r < (int64_t)nv;
         r += (int64_t)gridDim.x * 64) {
        const uint32_t j0 = off32[r];
        uint32_t j1 = r + 1 < (int64_t)nv ? off32[r + 1] : np;
        if (j1 > np) j1 = np;  // offsets are clamped to the capacity, n_pairs too
        // rows (index, wave) in index-major order form the range [j0 nq, j1 nq);
        // four loads are issued before they are added, in row order
        const int64_t k1 = (int64_t)j1 * nq;
        int64_t k = (int64_t)j0 * nq;
        float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
        for (; k + 4 <= k1; k += 4) {
            bool f[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) f[u] = flag[k + u] != 0;
            float4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (f[u]) v[u] = part[(k + u) * gs4 + c4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (f[u]) add4(a, v[u]);
            if (fifth) {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (f[u]) v[u] = part[(k + u) * gs4 + 4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (f[u]) add4(b, v[u]);
            }
        }
        for (; k < k1; ++k) {
            if (flag[k] == 0) continue;
            add4(a, part[k * gs4 + c4]);
            if (fifth) add4(b, part[k * gs4 + 4]);
        }
        float4 *dst = grad + (int64_t)sorted_entry[r] * gs4;
        dst[c4] = a;
        if (fifth) dst[4] = b;
    }
}

}  // namespace

bool tile_shape_supported(int tw, int th) {
    return (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 16 && th == 16) ||
           (tw == 32 && th == 8) || (tw == 32 && th == 32);
}

// Dispatch on the tile shape, the wave split (16x8, 16x16, 32x8) and the LDS
// batch depth D.
#define FM_DISPATCH(FN, D, ...)                                                                   \
    do {                                                                                          \
        if (p.tile_w == 16 && p.tile_h == 16)                                                     \
            return p.split ? FN<Geo<16, 16, true, D>>(__VA_ARGS__) : FN<Geo<16, 16, false, D>>(__VA_ARGS__); \
        if (p.tile_w == 8 && p.tile_h == 8) return FN<Geo<8, 8, false, D>>(__VA_ARGS__);           \
        if (p.tile_w == 16 && p.tile_h == 8)                                                      \
            return p.split ? FN<Geo<16, 8, true, D>>(__VA_ARGS__) : FN<Geo<16, 8, false, D>>(__VA_ARGS__); \
        if (p.tile_w == 32 && p.tile_h == 8)                                                      \
            return p.split ? FN<Geo<32, 8, true, D>>(__VA_ARGS__) : FN<Geo<32, 8, false, D>>(__VA_ARGS__); \
        if (p.tile_w == 32 && p.tile_h == 32) return FN<Geo<32, 32, false, D>>(__VA_ARGS__);       \
        return hipErrorInvalidValue;                                                              \
    } while (0)

hipError_t launch_render_fwd(const Plan &p, void *ws, const KParams &kp, const fm_outputs &out, hipStream_t st) {
    if (p.T == 0) return hipSuccess;
    FM_DISPATCH(fwd_t, 64, p, ws, kp, out, st);
}

hipError_t launch_render_bwd(const Plan &p, void *ws, const KParams &kp, const fm_outputs &out,
                             const fm_grad_outputs &g, hipStream_t st) {
    if (p.T == 0) return hipSuccess;
    FM_DISPATCH(bwd_t, 64, p, ws, kp, out, g, st);
}

hipError_t launch_render_fused(const Plan &p, void *ws, const KParams &kp, const LossArgs &la,
                               const fm_outputs &out, hipStream_t st) {
    if (p.T == 0) return hipSuccess;
    if (p.depth == 32) FM_DISPATCH(fused_t, 32, p, ws, kp, la, out, st);
    if (p.depth == 128) FM_DISPATCH(fused_t, 128, p, ws, kp, la, out, st);
    FM_DISPATCH(fused_t, 64, p, ws, kp, la, out, st);
}

hipError_t launch_render_prune(const Plan &p, void *ws, const KParams &kp, const PruneArgs &pa,
                               const fm_outputs &out, hipStream_t st) {
    if (p.T == 0) return hipSuccess;
    FM_DISPATCH(prune_t, 64, p, ws, kp, pa, out, st);
}

hipError_t launch_det_clear(const Plan &p, void *ws, int gstride, hipStream_t st) {
    (void)gstride;
    if (!p.det) return hipSuccess;
    const int64_t n4 = (p.cap * p.nq + 3) / 4;
    const int blocks = (int)std::min<int64_t>((n4 + 255) / 256, 2048);
    hipLaunchKernelGGL(k_det_clear, dim3(blocks), dim3(256), 0, st, at<uint32_t>(ws, p.o_pflag),
                       at<Status>(ws, p.o_status), p.nq);
    return hipGetLastError();
}

hipError_t launch_det_reduce(const Plan &p, void *ws, int gstride, hipStream_t st) {
    if (!p.det) return hipSuccess;
    // binning leaves the depth-ordered entries in the val buffer and their
    // pair offsets in the key buffer
    const int blocks = (int)std::min<int64_t>((p.E + 63) / 64, 16384);
    hipLaunchKernelGGL(k_det_reduce, dim3(blocks), dim3(256), 0, st, at<uint32_t>(ws, p.o_val),
                       at<uint32_t>(ws, p.o_key), at<Status>(ws, p.o_status), at<float4>(ws, p.o_part),
                       at<uint8_t>(ws, p.o_pflag), p.nq,
                       gstride / 4, at<float4>(ws, p.o_grad));
    return hipGetLastError();
}

hipError_t launch_loss_reduce(const Plan &p, void *ws, float *loss, hipStream_t st) {
    if (p.T == 0 || !loss) return hipSuccess;
    // one partial per block: a tile runs nq blocks
    const int64_t nb = p.T * p.nq;
    hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(1024), 0, st, at<float>(ws, p.o_loss), nb, loss,
                       (int)p.overwrite);
    return hipGetLastError();
}

}  // namespace fm
