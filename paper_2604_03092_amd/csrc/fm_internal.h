// fm_internal.h -- shared device-side layout of the gfx950 surfel rasterizer.
//
// Workspace organisation (one caller-owned device buffer, carved on the host
// by make_plan):
//   entries   one slot per (view, surfel of the view's submap); each view's
//             segment is padded to 256 so a 256-thread block never straddles
//             two views.  Per entry: an 80-byte projected record (Rec), a
//             32-bit depth key, a tile count, and a 64-byte gradient slot.
//   pairs     (global tile id, entry id), capacity max_pairs, double-buffered
//             for the radix sort.
//   tiles     per global tile [start, end) into the sorted pair list.
//   pixels    per pixel: final transmittance and the length of the prefix of
//             the tile list that the pixel composited.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fm2dgs.h"

namespace fm {

constexpr int kEntryAlign = 256;   // entry segment padding per view
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortBlock = 256;    // threads per radix-sort block
constexpr int kScanChunk = 2048;   // entries per block of the count scan
constexpr int kSortTile = 4096;     // items per block of a radix pass
constexpr int kEmitChunk = 2048;   // pairs per chunk of the emission blocks (two per sort tile)
constexpr int kMaxEmitGrid = 4096;
constexpr int kMaxPasses = 8;      // radix passes per binning (4 depth + up to 4 tile)

// Per-view descriptor, written into the workspace at the start of each call.
struct ViewDesc {
    const float *mean, *quat, *scale, *opacity, *color;  // the view's submap
    int32_t n;           // surfels in that submap
    int32_t submap;
    int32_t entry_base;  // first entry of the view (multiple of 256)
    int32_t width, height;
    int32_t tiles_x, tiles_y;
    int32_t tile_base;   // first global tile id
    int64_t pixel_offset;
    int32_t pad[2];
};

// Per-submap descriptor for the surfel-major backward projection.
struct SubmapDesc {
    const float *mean, *quat, *scale, *opacity, *color;
    float *g_mean, *g_quat, *g_scale, *g_opacity, *g_color;
    int32_t n;
    int32_t view_begin, view_count;  // slice of the submap-ordered view list
    int32_t block_base;              // first block of the backward projection
    int32_t proj_block_base;         // first block of the projection
};

// Projected surfel as the blend kernels consume it (80 bytes).
// With H = K [s_u t_u | s_v t_v | p] (columns) and its rows shifted to a
// pixel frame centred on (xs, ys): row0' = row0 - xs row2, row1' = row1 -
// ys row2, the pixel ray through (x, y) meets the surfel plane where
// (u, v, 1) ~ w = (row0' - x' row2) x (row1' - y' row2), x' = x - xs,
// y' = y - ys.  w is linear in the pixel coordinates:
//     w(x', y') = c0 + x' c2 - y' c1,
//     c0 = row0' x row1',  c1 = row0' x row2,  c2 = row1' x row2,
// so the blend kernels store the three vectors instead of H.
struct alignas(16) Rec {
    float c0[3], c1[3], c2[3];
    float sigma;
    float col[3];
    float nrm[3];   // camera-space unit normal facing the camera
    float z;        // camera-space depth of the centre
    float xs, ys;   // pixel-frame shift (integers, exact in float)
    float lsig;     // log2(sigma): sigma G = exp2(log2(sigma) - r^2 / (2 ln 2))
};
static_assert(sizeof(Rec) == 80, "record layout");

// Image-space support ellipse of one entry, used to cull 8x8 pixel blocks.
// The ellipse {p : (p - e)^T S^-1 (p - e) <= 1} (radius including the
// opacity cut-off and a small safety enlargement) is kept in the form the
// emission evaluates: centre (ex, ey), half-extents hx = sqrt(S00),
// hy = sqrt(S11), the slice at height dy spanning
// k1 dy +- sqrt(k2 (hy^2 - dy^2)) with k1 = S01 / S11, k2 = det S / S11^2,
// and dyr = S01 / hx, the height of its rightmost point (S in FP64, the
// derived values in FP32).  The entry's tile rect (from the canonical inclusive
// pixel-centre bbox) rides along: tb is the batch-global id of its top-left
// tile, t0 = tx0 | ty0 << 16 that tile's position in the view,
// nt = (tiles per rect row) | (tiles_x of the view) << 16.  Padded to 64
// bytes: the emission gathers the structs in depth order, and a 64-byte
// aligned struct never straddles two 128-byte cache lines.
struct alignas(64) Ell {
    float ex, ey, hx, hy;
    float k1, k2, dyr;
    uint32_t tb;
    uint32_t t0, nt, pad[6];
};
static_assert(sizeof(Ell) == 64, "ellipse layout");

// Pair values: entry id in the low 28 bits, 8x8-block mask of the tile in the
// high 4 bits (bit b set when block b of the tile may hold a covered pixel);
// for 32x32 tiles the bits mark 16x16 quadrants.
constexpr uint32_t kEntryMask = 0x0FFFFFFFu;
constexpr int kMaskShift = 28;

// Gradient slot of one entry: dL/dc0[3], dL/dc1[3], dL/dc2[3], dL/dsigma,
// dL/dcol[3], dL/dz, then dL/dn[3] when the normal map carries a gradient.
// Slots are kGradSlot = 16 floats (64 bytes, two per 128-byte cache line:
// zeroing and the blend's atomics touch one line per slot) when it does not
// (the fused L1 path) and kGradStride = 20 floats when it does.
constexpr int kGradStride = 20;
constexpr int kGradSlot = 16;

struct Status {
    uint32_t n_pairs;    // pairs actually stored (min(required, capacity))
    uint32_t overflow;   // 1 when required > capacity
    uint64_t required;   // pairs the batch needs
    uint32_t n_vis;      // entries that cover at least one tile
    uint32_t n_kept;     // pairs in the tile-sorted list (those of tiles the support reaches)
    uint32_t pad[2];
};

struct KParams {
    float alpha_min, alpha_max, t_min, rho_max, near_plane;
    float bg[3];
    int32_t tile_w, tile_h;
    int32_t gstride;  // floats per gradient slot: kGradSlot, or kGradStride with normal gradients
    uint32_t pair_cap;  // pair capacity (bounds the emission indices of deterministic lists)
};

struct LossArgs {
    const float *target_rgb, *target_depth;
    const uint8_t *mask;
    float w_rgb, w_depth;
};

// Map-fusion pruning: the error criterion's inputs, or a caller mask.
struct PruneArgs {
    const float *target_rgb, *target_depth;
    const uint8_t *mask_in;
    uint8_t *mask_out;
    float tau_rgb, tau_depth;
};

struct Plan {
    int V = 0, S = 0;
    int64_t E = 0;      // entries (padded)
    int64_t T = 0;      // total tiles
    int64_t NPX = 0;    // total pixels
    int64_t cap = 0;    // pair capacity
    int max_view_entries = 0;
    int tile_w = 16, tile_h = 16;
    int tile_bits = 1;
    int pair_passes = 1;
    int sortG_e = 1, sortG_p = 1;
    int scan_blocks = 1;
    int emit_blocks = 1;
    int proj_blocks = 0;    // total blocks of the projection (surfel blocks x view groups per submap)
    int a7_blocks = 0;      // total blocks of the backward projection
    int a7_max_blocks = 0;  // max blocks of one submap
    size_t o_views = 0, o_subs = 0, o_vlist = 0, o_status = 0, o_rec = 0, o_key = 0, o_cnt = 0,
           o_key2 = 0, o_val = 0, o_val2 = 0, o_scan = 0, o_pkey = 0, o_pval = 0, o_pkey2 = 0,
           o_pval2 = 0, o_hist = 0, o_tstart = 0, o_tend = 0, o_tfinal = 0, o_nlast = 0, o_ncount = 0, o_grad = 0,
           o_pose = 0, o_loss = 0, o_tot = 0, o_ell = 0, o_chunk = 0, o_meta = 0, o_part = 0,
           o_torder = 0, o_emeta = 0, o_tbucket = 0, o_cnt2 = 0, o_cnt3 = 0, o_pflag = 0;
    size_t bytes = 0;
    // deterministic gradients: the sorted lists hold emission indices, o_meta
    // maps them to pair values, and the adjoint writes one partial slot per
    // (pair, wave of the tile) at o_part and sets its byte at o_pflag; the
    // flagged slots are summed per entry in emission order
    bool det = false;
    bool overwrite = false;  // store (not add) surfel gradients, pose gradients and the loss
    bool lpt = true;         // blend takes tiles longest list first (else image order)
    int nq = 1;  // waves (blocks of the blend) per tile: four 16x16 quadrants of a 32x32 tile, one per 8x8 block with split
    bool split = false;  // 16x8, 16x16, 32x8 tiles: one blend wave per 8x8 block instead of one per tile
    int depth = 64;      // records the fused blend stages in LDS per batch (32, 64 or 128)
    bool pairs_in_alt = false;  // final sorted pairs live in the *2 buffers
};

template <class T> __host__ __device__ inline T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// Index of the last view whose `entry_base` (or `tile_base`) is <= x.
__device__ inline int view_of_entry(const ViewDesc *v, int V, int64_t x) {
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if ((int64_t)v[mid].entry_base <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}
__device__ inline int view_of_tile(const ViewDesc *v, int V, int64_t x) {
    int lo = 0, hi = V - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if ((int64_t)v[mid].tile_base <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Workgroups are dealt to the 8 XCDs of the chip round-robin.  Remapping
// workgroup b of n to logical index (b mod 8) * (n / 8) + b / 8 gives every
// XCD a contiguous run of logical indices (the tail beyond a multiple of 8
// maps to itself), so neighbouring tiles or chunks share one L2.
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t n) {
    const uint32_t per = n >> 3;
    return b < per * 8u ? (b & 7u) * per + (b >> 3) : b;
}

// The same at a finer grain: within every group of 8 C consecutive
// workgroups, each XCD gets C consecutive logical indices (tail unchanged).
// Neighbouring tiles still meet in one L2, while every XCD keeps sampling
// the whole batch (a contiguous 1/8 of it can cost more than another).
template <uint32_t C> __device__ __forceinline__ uint32_t xcd_chunked(uint32_t b, uint32_t n) {
    constexpr uint32_t grp = 8u * C;
    return b < (n / grp) * grp ? (b / grp) * grp + (b & 7u) * C + (b >> 3) % C : b;
}

// Start of a call's binning state, run by every block of a 256-thread grid:
// block 0 clears the status words and the blend order's bucket counts and
// cursors, and the grid starts every tile range empty with ts > te (the last
// tile-sort pass fills the ranges).  The setup kernels run it, before the
// projection (which touches none of it).
__device__ __forceinline__ void init_ranges_block(uint32_t *status, int n_status, uint32_t *tbucket,
                                                  uint32_t *ts, uint32_t *te, int64_t n) {
    if (blockIdx.x == 0 && (int)threadIdx.x < n_status) status[threadIdx.x] = 0u;
    if (blockIdx.x == 0) {
        tbucket[threadIdx.x] = 0u;
        tbucket[kRadix + threadIdx.x] = 0u;
    }
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        ts[i] = 0xFFFFFFFFu;
        te[i] = 0u;
    }
}

// ---- launchers (host) ------------------------------------------------------
// start_binning: also start the binning state of a call that bins (forward,
// fused, pruning), not of a backward that reads a previous forward's lists
hipError_t launch_setup(const Plan &p, void *ws, const ViewDesc *views, const SubmapDesc *subs,
                        const int32_t *vlist, bool start_binning, hipStream_t st);
// views one projection thread handles
constexpr int kProjViewsPerThread = 4;
hipError_t launch_preprocess(const Plan &p, void *ws, const KParams &kp, const float *intr,
                             const float *viewmat, bool zero_grad, hipStream_t st);
hipError_t launch_binning(const Plan &p, void *ws, hipStream_t st);
// the binning state's start (init_ranges_block) as a kernel of its own
hipError_t launch_init_ranges(const Plan &p, void *ws, hipStream_t st);
int init_ranges_blocks(const Plan &p);
hipError_t launch_render_fwd(const Plan &p, void *ws, const KParams &kp, const fm_outputs &out,
                             hipStream_t st);
hipError_t launch_render_bwd(const Plan &p, void *ws, const KParams &kp, const fm_outputs &out,
                             const fm_grad_outputs &g, hipStream_t st);
hipError_t launch_render_fused(const Plan &p, void *ws, const KParams &kp, const LossArgs &la,
                               const fm_outputs &out, hipStream_t st);
hipError_t launch_loss_reduce(const Plan &p, void *ws, float *loss, hipStream_t st);
// Pruning products: forward render, error flags and per-entry scores (the
// first float of each entry's gradient slot, cleared by the projection), then
// the per-surfel sum over the views (into each submap's g_opacity pointer).
hipError_t launch_render_prune(const Plan &p, void *ws, const KParams &kp, const PruneArgs &pa,
                               const fm_outputs &out, hipStream_t st);
hipError_t launch_score_reduce(const Plan &p, void *ws, int gstride, hipStream_t st);
// Removal of the surfels whose score exceeds tau (order kept).
size_t prune_compact_workspace_bytes(int64_t n);
hipError_t launch_prune_compact(const fm_surfels &in, const float *score, float tau, const fm_surfel_buffer &out,
                                int32_t *count, void *ws, hipStream_t st);
hipError_t launch_zero_grad(const Plan &p, void *ws, int gstride, hipStream_t st);
// Deterministic gradients: clear the partial slots of the stored pairs before
// an adjoint, and sum each entry's slots into its gradient slot after it.
hipError_t launch_det_clear(const Plan &p, void *ws, int gstride, hipStream_t st);
hipError_t launch_det_reduce(const Plan &p, void *ws, int gstride, hipStream_t st);
hipError_t launch_preprocess_bwd(const Plan &p, void *ws, int gstride, const float *intr, const float *viewmat,
                                 float *dL_dviewmat, hipStream_t st);
bool tile_shape_supported(int tw, int th);
// LDS read probe of the benchmark (mode 0: per-lane words, 1: wave broadcast)
hipError_t launch_lds_probe(int mode, int blocks, int iters, float *sink, hipStream_t st);
int64_t lds_probe_bytes(int blocks, int iters);
size_t fusion_workspace_bytes(int32_t width, int32_t height);
size_t fusion_batch_workspace_bytes(const fm_pixel_map *maps, int32_t n);
hipError_t launch_fusion_batch(const fm_pixel_map *maps, const fm_sim3 *poses, int32_t n,
                               const fm_fusion_params &fp, const float *const *accums, const fm_surfel_buffer &out,
                               int32_t *offsets, int32_t *total, void *ws, hipStream_t st);
hipError_t launch_fusion(const fm_pixel_map &in, const fm_sim3 &pose, const fm_fusion_params &fp,
                         const float *accum, const fm_surfel_buffer &out, int32_t *count, void *ws,
                         hipStream_t st);
hipError_t launch_warp(float *mean, float *quat, float *scale, const int32_t *kf, int64_t n,
                       const fm_sim3 *deltas, int32_t K, hipStream_t st);
hipError_t launch_adam(const fm_adam_tensor *ts, int count, const fm_adam_config &cfg, int32_t *step,
                       hipStream_t st);

}  // namespace fm
