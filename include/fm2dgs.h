/*
 * fm2dgs.h -- C ABI of the MI355X (gfx950) differentiable 2D Gaussian surfel
 * rasterizer: the data-parallel hot path of the 2DGS mapping backend of
 * Flash-Mono (arXiv 2604.03092).
 *
 * What is computed.  A surfel map (per surfel: centre mu, colour c, opacity
 * sigma, rotation r as a quaternion, two tangent scales s; Sec. 3,
 * "Preliminaries") is seen from one or more pinhole cameras.  Each pixel
 * composites the surfels that cover it front to back with the volumetric
 * alpha blending of Eq. 1: (I, D, A) = sum_i (c_i, z_i, 1) w_i prod_{j<i}
 * (1 - w_j), plus a camera-space normal map sum_i n_i w_i prod_{j<i}(1-w_j).
 * The weight w_i is evaluated by exact ray-splat intersection (the surfel is
 * a planar disk, Sec. 3): the pixel ray meets the surfel plane at local
 * coordinates (u, v), G = exp(-(u^2+v^2)/2), w_i = alpha_i =
 * min(alpha_max, sigma_i G); a surfel is skipped at a pixel when
 * u^2 + v^2 > rho_max^2 or sigma_i G < alpha_min, and compositing stops
 * before the surfel that would take the transmittance below t_min.  z_i is
 * the camera-space depth of the surfel centre, n_i the camera-space surfel
 * normal turned to face the camera.  Surfels with equal depth key are taken
 * in index order.  The image adds T_final * background.
 *
 * The backward returns dL/d(mean, quat, scale, opacity, color) of every
 * surfel and dL/d(view matrix) of every view, given dL/d(outputs).  The
 * fused call evaluates the backend's L1 render loss (Sec. 3.1 render term,
 * refinement of Sec. 3.3) and its gradient in one pass.
 *
 * Conventions (all calls):
 *   - Every pointer inside fm_surfels, fm_outputs, fm_grad_outputs,
 *     fm_surfel_grads, the intrinsics/view-matrix arrays, targets, masks,
 *     the loss scalar and the workspace is DEVICE memory owned by the
 *     caller.  fm_batch.submaps and fm_batch.views are HOST arrays.
 *   - Planes are float32, structure-of-arrays, channel-major.  Per-pixel
 *     planes cover all views of a batch back to back, view v starting at
 *     sum_{u<v} W_u H_u, rows top to bottom, pixel (col,row) has its centre
 *     at (col+0.5, row+0.5).
 *   - Quaternions are (w,x,y,z) of any non-zero norm (normalised inside;
 *     gradients are w.r.t. the raw values).  Scales are linear and > 0;
 *     opacity is the activated value.  Activations belong to the caller.
 *   - intr[v] = (fx, fy, cx, cy); viewmat[v] = world->camera [R|t], 12
 *     floats row-major.  A Sim(3) keyframe pose renders as its SE(3) part
 *     with depths divided by the scale; that scaling is the caller's.
 *   - Gradients are ACCUMULATED (+=) into the caller's buffers, or stored
 *     when params->overwrite is 1.
 *   - Surfels with any non-finite value, a zero quaternion, a non-positive
 *     scale, depth <= near_plane, opacity <= alpha_min, or a support disk
 *     not entirely in front of the camera are culled: they contribute
 *     nothing and receive zero gradient.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = default stream)
 *     and the calls return without synchronising.  No call allocates
 *     device memory or synchronises except fm_create, fm_query_status,
 *     fm_debug_pairs and fm_autotune, so fm_forward, fm_backward and
 *     fm_fwd_bwd_l1 may be captured into a HIP graph.
 *   - Errors: every call returns an fm_status and never throws.  Arguments
 *     are validated on the host before anything is launched; on failure
 *     nothing is enqueued and fm_last_error(ctx) describes the problem.
 *   - Calls on one fm_ctx are not thread-safe.
 */
#ifndef FM2DGS_H
#define FM2DGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int fm_status;
#define FM_OK 0
#define FM_ERR_INVALID_ARG 1   /* bad pointer, size, index or parameter          */
#define FM_ERR_CAPACITY 2      /* pair buffer too small (see fm_query_status)     */
#define FM_ERR_HIP 3           /* a HIP runtime call failed                       */
#define FM_ERR_UNSUPPORTED 4   /* e.g. a tile shape the library was not built for */
#define FM_ERR_WORKSPACE 5     /* workspace smaller than fm_workspace_size        */

typedef struct fm_ctx fm_ctx;

/* One surfel map (a submap).  Device pointers, float32, n surfels:
 * mean[3][n], quat[4][n] (w,x,y,z), scale[2][n], opacity[n], color[3][n]. */
typedef struct {
    int32_t n;
    const float *mean;
    const float *quat;
    const float *scale;
    const float *opacity;
    const float *color;
} fm_surfels;

/* Gradient buffers of one submap, same layout as fm_surfels; += semantics.
 * A NULL member skips that gradient. */
typedef struct {
    float *mean;
    float *quat;
    float *scale;
    float *opacity;
    float *color;
} fm_surfel_grads;

/* One view (host struct): image size and the submap it renders. */
typedef struct {
    int32_t width;   /* 1 .. 16384 */
    int32_t height;  /* 1 .. 16384 */
    int32_t submap;  /* index into fm_batch.submaps */
} fm_view_shape;

/* A batch: several views over one or several submaps (Sec. 3.3 refines the
 * latest keyframes; each keyframe is a view). */
typedef struct {
    int32_t n_submaps;
    const fm_surfels *submaps;   /* HOST array [n_submaps] */
    int32_t n_views;
    const fm_view_shape *views;  /* HOST array [n_views] */
    const float *intr;           /* DEVICE [n_views][4]  fx, fy, cx, cy */
    const float *viewmat;        /* DEVICE [n_views][12] world->camera [R|t] */
} fm_batch;

/* Rasterization parameters; fm_default_params fills the defaults. */
typedef struct {
    float alpha_min;   /* 1/255: skip a surfel at a pixel when sigma G < alpha_min
                          (>= 1e-6, so every composited surfel lowers T)         */
    float alpha_max;   /* 0.99: clamp of alpha (must be < 1 for the backward)     */
    float t_min;       /* 1e-4: stop before the transmittance would fall below it
                          (>= 1e-30)                                             */
    float rho_max;     /* 3: support radius in units of the tangent scales        */
    float near_plane;  /* 0.2: cull surfels with centre depth <= near_plane       */
    float bg[3];       /* background colour added with weight T_final             */
    int32_t tile_w;    /* tile shape in pixels: 8x8, 16x8, 16x16, 32x8 or 32x32    */
    int32_t tile_h;    /* (rendered as four 16x16 quadrants sharing one list);
                          0x0 uses the context's autotuned choice for the batch,
                          else 16x16                                            */
    int32_t deterministic;  /* 0: per-entry gradients are summed with float atomics in
                               the order tiles finish (equal between runs up to
                               rounding).  1: every (pair, wave) writes its own
                               partial and each entry sums its partials in emission
                               order, so gradients, the pose gradient and the loss are
                               bitwise reproducible; the workspace grows by
                               4 + 81 * w bytes per pair of capacity (w = waves per
                               tile: 4 for 32x32, the 8x8 blocks of the tile with
                               tile_waves 2, else 1: a partial slot and a written
                               flag per wave) and a step costs one clear of the
                               flags and one reduction pass over the written
                               partials.  Forward,
                               backward and fwd_bwd calls on one workspace must agree
                               on it.  Other values are INVALID_ARG.               */
    int32_t overwrite;      /* 0: surfel gradients, dL_dviewmat and the fused call's
                               loss are ADDED into the caller's buffers.  1: they
                               are STORED, so nothing needs clearing beforehand:
                               every element of a submap that some view of the
                               batch renders, every view's dL_dviewmat row and
                               *loss are overwritten; submaps that no view renders
                               are left untouched.  Other values are INVALID_ARG. */
    int32_t tile_order;     /* order in which the blend takes the tiles: 1 = longest
                               list first (long tiles start early and short ones
                               fill the end of the launch); 2 = image order
                               (neighbouring tiles run together and share surfel
                               records in cache); 0 = the order fm_autotune chose
                               for this batch and tile shape, else 1.  It changes
                               only the schedule: forward and backward calls on one
                               workspace may differ in it.  Other values are
                               INVALID_ARG.                                        */
    int32_t tile_waves;     /* work split of the blend: 1 = one wave per tile (four
                               16x16 quadrant waves for 32x32 tiles); 2 = one wave
                               per 8x8 block of a 16x8, 16x16 or 32x8 tile, which
                               traverse the tile's one list side by side (more,
                               shorter waves for batches that do not fill the
                               chip; 8x8 and 32x32 tiles are the same either
                               way); 0 = fm_autotune's choice for this batch and
                               tile shape, else 1.  It changes only the schedule:
                               images are bitwise the same.  With deterministic
                               sums, forward, backward and fwd_bwd calls on one
                               workspace must agree on it (the partial gradient
                               slots are per wave).  Other values are INVALID_ARG. */
    int32_t lds_depth;      /* surfel records the fused call's blend stages in LDS
                               per batch: 32, 64 or 128; 0 = fm_autotune's choice
                               for this batch and tile shape, else 64.  The other
                               calls stage 64.  Deterministic sums need 64 (or 0).
                               Other values are INVALID_ARG.                      */
} fm_raster_params;

/* Output planes (device, float32): rgb[3][P], depth[P], normal[3][P],
 * alpha[P], P = total pixels of the batch.  Depth and normal are the
 * unnormalised sums of Eq. 1 (divide by alpha for a mean). */
typedef struct {
    float *rgb;
    float *depth;
    float *normal;
    float *alpha;
} fm_outputs;

/* Upstream gradients dL/d(outputs), same layout.  A NULL member means zero. */
typedef struct {
    const float *rgb;
    const float *depth;
    const float *normal;
    const float *alpha;
} fm_grad_outputs;

/* L1 render loss of the fused call: for every view v with P_v pixels,
 *   L += w_rgb   * sum_px mask * |I - I*| / (3 P_v)
 *      + w_depth * sum_px mask * |D - D*| / P_v
 * target_rgb[3][P], target_depth[P] (may be NULL when w_depth == 0),
 * mask[P] as uint8 0/1 (NULL = all ones).  sign(0) = 0. */
typedef struct {
    const float *target_rgb;
    const float *target_depth;
    const uint8_t *mask;
    float w_rgb;
    float w_depth;
} fm_l1_loss;

/* Context: binds to a HIP device, queries its properties and holds the
 * autotuner's choices.  Allocates no device memory; the first context on a
 * device resolves that device's address of the static scratch array of
 * fm_fwd_bwd_l1_noalloc. */
fm_status fm_create(fm_ctx **ctx, int device);
void fm_destroy(fm_ctx *ctx);
const char *fm_status_string(fm_status s);
const char *fm_last_error(const fm_ctx *ctx);
void fm_default_params(fm_raster_params *p);
/* Library version as major*10000 + minor*100 + patch. */
int fm_version(void);

/* Bytes of workspace a batch needs with room for max_pairs (surfel, tile)
 * pairs.  The workspace holds the projected surfels, the sorted pair list,
 * per-pixel saved state and gradient scratch; it must stay untouched from
 * fm_forward until the matching fm_backward has run. */
fm_status fm_workspace_size(fm_ctx *ctx, const fm_batch *batch, const fm_raster_params *params,
                            int64_t max_pairs, size_t *bytes);

/* Forward render of every view of the batch into `out`.  If more than
 * max_pairs pairs are needed the extra pairs are dropped (nothing is written
 * out of bounds), the workspace records the overflow and fm_query_status
 * reports FM_ERR_CAPACITY with the required count. */
fm_status fm_forward(fm_ctx *ctx, const fm_batch *batch, const fm_raster_params *params,
                     fm_outputs out, void *workspace, size_t ws_bytes, int64_t max_pairs,
                     void *stream);

/* Backward of the preceding fm_forward on the same workspace, batch and
 * parameters.  `out` must still hold that forward's outputs (they enter the
 * adjoint of the compositing).  grads is a HOST array [n_submaps];
 * dL_dviewmat (device, [n_views][12], may be NULL) receives dL/d[R|t]. */
fm_status fm_backward(fm_ctx *ctx, const fm_batch *batch, const fm_raster_params *params,
                      fm_outputs out, fm_grad_outputs dL_dout, void *workspace, size_t ws_bytes,
                      int64_t max_pairs, const fm_surfel_grads *grads, float *dL_dviewmat,
                      void *stream);

/* Fused forward + L1 loss + backward of the whole batch (the refinement
 * step's render term, Sec. 3.3).  Writes the outputs, ADDS the loss into
 * *loss (device float; stores it with params->overwrite) and accumulates
 * (or stores) the gradients as fm_backward does. */
fm_status fm_fwd_bwd_l1(fm_ctx *ctx, const fm_batch *batch, const fm_raster_params *params,
                        const fm_l1_loss *loss_spec, fm_outputs out, float *loss,
                        const fm_surfel_grads *grads, float *dL_dviewmat, void *workspace,
                        size_t ws_bytes, int64_t max_pairs, void *stream);

/* For callers that cannot allocate (code under HIP graph capture without a
 * workspace of its own, tight serving loops, harnesses that forbid
 * allocation): fm_fwd_bwd_l1 with its workspace taken from a static device
 * array of FM_NOALLOC_SCRATCH_BYTES (128 MiB) that the library keeps on each
 * GPU it runs on until the process ends (its device address is resolved by
 * fm_create).  Same arguments and results as fm_fwd_bwd_l1 without the
 * workspace.  A batch whose workspace (fm_workspace_size with this
 * max_pairs) exceeds FM_NOALLOC_SCRATCH_BYTES fails with FM_ERR_WORKSPACE
 * before anything is enqueued; the 640x480 view of 300k surfels fits with
 * room for 1.5M pairs.  Every call on one GPU uses that GPU's one array,
 * which keeps the last call's contents: calls that overlap on one GPU (other
 * streams, contexts or host threads) race and give wrong results, so the
 * caller serialises them.  pair_status (device, 2 int64, may be NULL)
 * receives the pairs the batch needed and 1 if that exceeded max_pairs
 * (the results are then incomplete, as with FM_ERR_CAPACITY), else 0.
 * Calls no allocating routine and does not synchronise. */
#define FM_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
fm_status fm_fwd_bwd_l1_noalloc(fm_ctx *ctx, const fm_batch *batch, const fm_raster_params *params,
                                const fm_l1_loss *loss_spec, fm_outputs out, float *loss,
                                const fm_surfel_grads *grads, float *dL_dviewmat, int64_t max_pairs,
                                int64_t *pair_status, void *stream);

/* After the stream that ran fm_forward / fm_fwd_bwd_l1 has been synchronised:
 * reads the pair count of the last forward on this workspace.  Returns
 * FM_ERR_CAPACITY (and the required count) if the pair buffer overflowed,
 * else FM_OK.  Synchronous device read. */
fm_status fm_query_status(fm_ctx *ctx, const fm_batch *batch, const fm_raster_params *params,
                          const void *workspace, int64_t max_pairs, int64_t *n_pairs,
                          int64_t *required_pairs);

/* Test hook: copies the sorted pair list of the last forward into HOST
 * buffers (cap entries each): tile[k] = global tile id (views' tiles back to
 * back, row-major within a view), entry[k] = view-local surfel index, view[k]
 * = view index, and the per-tile ranges tile_start/tile_end (host arrays
 * sized to the batch's total tile count; 0, 0 for a tile without pairs).  *n_pairs is the length of the
 * list: the pairs of each surfel's tile rect (the count fm_query_status
 * reports) less those of tiles that its opacity-cut support ellipse,
 * conservatively enlarged, does not reach.  Synchronous. */
fm_status fm_debug_pairs(fm_ctx *ctx, const fm_batch *batch, const fm_raster_params *params,
                         const void *workspace, int64_t max_pairs, uint32_t *tile,
                         uint32_t *surfel, uint32_t *view, int64_t cap, int64_t *n_pairs,
                         uint32_t *tile_start, uint32_t *tile_end, int64_t n_tiles);

/* Test hook: copies the per-pixel final transmittance and number of
 * composited surfels into HOST buffers of npx entries (npx >= total pixels
 * of the batch).  The transmittance is the last fm_forward's or
 * fm_fwd_bwd_l1's; the counts are written by fm_forward only (the fused
 * path does not count).  Synchronous. */
fm_status fm_debug_pixel_state(fm_ctx *ctx, const fm_batch *batch, const fm_raster_params *params,
                               const void *workspace, int64_t max_pairs, float *t_final,
                               uint32_t *n_contrib, int64_t npx);

/* Test and benchmark hook: counts of the last forward on this workspace,
 * read after the stream has been synchronised: *n_visible = (view, surfel)
 * entries whose tile rect is not empty, *n_kept = pairs in the tile-sorted
 * list (either pointer may be NULL).  Synchronous. */
fm_status fm_debug_counts(fm_ctx *ctx, const fm_batch *batch, const fm_raster_params *params,
                          const void *workspace, int64_t max_pairs, int64_t *n_visible,
                          int64_t *n_kept);

/* Benchmark hook, not part of rendering: LDS read bandwidth of the device.
 * Enqueues `blocks` workgroups of 256 threads; every thread reads 16-byte
 * words from LDS 8 * iters times and stores one float into sink (device,
 * blocks * 256 floats).  mode 0: each lane its own word, consecutive lanes
 * consecutive words (no bank conflicts); mode 1: all lanes of a wave the same
 * word (a broadcast, the blend kernels' access to staged records).
 * *lane_bytes (host, may be NULL) receives the bytes delivered to lanes,
 * blocks * 256 * 8 * iters * 16.  The caller times the stream. */
fm_status fm_bench_lds(fm_ctx *ctx, int32_t mode, int32_t blocks, int32_t iters, float *sink,
                       double *lane_bytes, void *stream);

/* Benchmark hook.  With timing enabled, fm_forward / fm_backward /
 * fm_fwd_bwd_l1 record HIP events between their phases on the call's stream
 * (skipped while the stream is being captured).  fm_phase_times waits for the
 * last call's events and writes per-phase milliseconds into ms[0..5]:
 * 0 projection, 1 binning (depth sort, emission, tile sort, ranges),
 * 2 zeroing of gradient slots, 3 blend kernel (forward, backward or fused),
 * 4 loss reduction, 5 backward projection and pose reduction.  n >= 6. */
fm_status fm_set_timing(fm_ctx *ctx, int enable);
fm_status fm_phase_times(fm_ctx *ctx, float *ms, int n);

/* Total tile count of a batch for the given tile shape. */
fm_status fm_tile_count(const fm_batch *batch, const fm_raster_params *params, int64_t *n_tiles);

/* Autotuner: times fm_fwd_bwd_l1 in two stages, every call's status
 * checked and every call timed on its own (a candidate's score is its
 * median call after a warm-up call).  Stage 1, 5 calls each: the supported
 * tile shapes, each with both tile orders and, for tiles of several 8x8
 * blocks, both work splits (tile_waves 1 and 2), at LDS depth 64.  Stage 2,
 * 15 calls each: the default launch (16x16, tile_order 1, tile_waves 1,
 * depth 64) and the three fastest of stage 1, each at LDS depths 64, 32 and
 * 128 (depth 64 only with deterministic sums), in that order; a candidate
 * replaces the best so far only when its median is more than 1% lower.
 * Runs on this batch (outputs, gradients and the loss are
 * overwritten/accumulated while it runs), and
 * writes the stage-2 winner into *chosen (a copy of *params with
 * tile_w, tile_h, tile_order, tile_waves and
 * lds_depth set).  The choice is cached in the context under the device's
 * architecture, the batch's shape signature and the deterministic flag (the
 * two modes tune separately) and, if cache_path is not NULL, in a JSON file
 * read back by later contexts.  Shapes whose workspace (fm_workspace_size) exceeds
 * ws_bytes or whose pairs exceed max_pairs are skipped; without
 * deterministic sums the 8x8 workspace is the largest.  Synchronous. */
fm_status fm_autotune(fm_ctx *ctx, const fm_batch *batch, const fm_raster_params *params,
                      const fm_l1_loss *loss_spec, fm_outputs out, float *loss,
                      const fm_surfel_grads *grads, float *dL_dviewmat, void *workspace,
                      size_t ws_bytes, int64_t max_pairs, const char *cache_path,
                      fm_raster_params *chosen, void *stream);

/* ---- map refinement: optimizer step -------------------------------------
 *
 * The backend refines the map by gradient steps on the render loss
 * (Sec. 3.3).  The paper names no optimizer; fm_adam_step is Adam as defined
 * by Kingma & Ba (2015, Algorithm 1): with g the gradient of the tensor's
 * free variable theta, m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
 * theta <- theta - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * The rasterizer takes activated values p (opacity in (0, 1], linear scales),
 * so each tensor names the parameterisation theta(p) its step is taken in;
 * the kernel maps p and dL/dp to theta and dL/dtheta and maps the result
 * back into p. */
#define FM_PARAM_LINEAR 0  /* theta = p                                           */
#define FM_PARAM_LOG 1     /* theta = log p; p is first raised to >= 1e-30       */
#define FM_PARAM_LOGIT 2   /* theta = log(p / (1 - p)); p is first clamped into
                              [1e-6, 1 - 1e-6]                                    */

typedef struct {
    float *param;        /* DEVICE [n] activated values p, updated in place      */
    float *grad;         /* DEVICE [n] dL/dp (e.g. the fm_surfel_grads planes);   
                            read, and cleared when the config asks for it         */
    float *m;            /* DEVICE [n] first moment of theta (zero before step 1) */
    float *v;            /* DEVICE [n] second moment of theta (zero before step 1) */
    int64_t n;           /* elements (0: the tensor is skipped)                   */
    float lr;            /* learning rate of this tensor (> 0)                    */
    int32_t kind;        /* FM_PARAM_*                                            */
} fm_adam_tensor;

typedef struct {
    float beta1;         /* 0.9, in [0, 1)                                       */
    float beta2;         /* 0.999, in [0, 1)                                     */
    float eps;           /* 1e-8, > 0                                            */
    int32_t zero_grad;   /* non-zero: clear each gradient element after using it,
                            ready for the next accumulation                      */
} fm_adam_config;

/* One Adam step over count tensors (HOST array of descriptors), all tensors
 * in one launch (plus the counter's).  step is a
 * DEVICE int32 step counter: the call first advances it by one and every
 * update uses the advanced value t in its bias corrections, so a captured
 * graph replays consecutive steps.  The caller owns every buffer; tensors
 * must not overlap.  Enqueued on stream; no allocation, no synchronisation;
 * graph-capturable.  Errors: FM_ERR_INVALID_ARG for a NULL context, step or
 * descriptor array (count > 0), a negative count or n, n >= 2^31, NULL
 * buffers with n > 0, lr <= 0 or non-finite, an unknown kind, or betas outside [0, 1) or
 * eps <= 0; nothing is launched then.  FM_ERR_HIP if a launch fails. */
fm_status fm_adam_step(fm_ctx *ctx, const fm_adam_tensor *tensors, int32_t count, const fm_adam_config *config,
                       int32_t *step, void *stream);

/* ---- map fusion: an incoming per-pixel map -------------------------------
 *
 * The frontend predicts one surfel per pixel of a keyframe.  Before it joins
 * the global map (Sec. 3.3), the map is thinned by adaptive voxelization:
 * the pixel grid is cut into 2x2 blocks (blocks cut by the image border hold
 * 2 or 1 pixels); a block whose camera-space depth range max z - min z is at
 * most tau_depth becomes one primitive with the mean centre, scales, opacity
 * and colour of its pixels and the normalised sum of their quaternions, each
 * first sign-aligned with the block's first (Eq. for r_merged).  Blocks with
 * a larger depth range, and 1-pixel blocks, keep their primitives.  The
 * survivors move to world coordinates by the keyframe's similarity:
 * mu_w = s R(q) mu + t, r_w = q r (Hamilton product), scales times s.  With
 * an accumulation map (the accumulated alpha of the global map rendered from
 * the keyframe), primitives are only added where the map is not yet well
 * reconstructed: a merged block when the mean of its pixels' values is below
 * tau_accum, a kept pixel when its own value is.  The float comparisons are
 * made in float32 in the order: depth range as (max - min); accumulation
 * sum as (a0 + a1) + (a2 + a3) or a0 + a1, compared with tau_accum * n. */
typedef struct {
    int32_t width, height;  /* pixel grid (>= 1 each, width * height < 2^31)      */
    const float *mean;      /* DEVICE [3][W*H] camera-space centres, pixels row-major */
    const float *quat;      /* DEVICE [4][W*H] (w, x, y, z) rotations              */
    const float *scale;     /* DEVICE [2][W*H]                                      */
    const float *opacity;   /* DEVICE [W*H]                                         */
    const float *color;     /* DEVICE [3][W*H]                                      */
} fm_pixel_map;

typedef struct {
    float s;      /* scale (> 0)                                  */
    float q[4];   /* rotation (w, x, y, z), any non-zero norm     */
    float t[3];   /* translation                                  */
} fm_sim3;        /* camera -> world: x_w = s R(q) x_c + t         */

typedef struct {
    float tau_depth;  /* merge a block when its depth range is <= tau_depth (< 0: never)  */
    float tau_accum;  /* with an accumulation map: add only below this accumulated alpha */
} fm_fusion_params;

typedef struct {
    float *mean, *quat, *scale, *opacity, *color;  /* DEVICE [C][capacity] output planes */
    int64_t capacity;                              /* primitives the planes hold (>= 0)  */
} fm_surfel_buffer;

/* Workspace bytes fm_voxelize_fuse needs for a width x height map. */
size_t fm_fusion_workspace_size(int32_t width, int32_t height);

/* Voxelize, transform and gate one per-pixel map; the survivors are written
 * to out in block order (blocks row-major over the block grid, a kept
 * block's pixels row-major) and their number to *count (DEVICE int32).
 * Primitives beyond out.capacity are not written; *count still reports how
 * many there are, so a caller compares it with the capacity (width * height
 * always suffices).  accum: DEVICE [W*H] or NULL (no gate).  pose: HOST.
 * Enqueued on stream; no allocation, no synchronisation; graph-capturable.
 * Errors: FM_ERR_INVALID_ARG for NULL pointers, a grid outside the limits,
 * s <= 0, a zero or non-finite quaternion, a negative capacity or NULL output
 * planes with capacity > 0; FM_ERR_WORKSPACE when ws_bytes is below
 * fm_fusion_workspace_size; FM_ERR_HIP if a launch fails. */
fm_status fm_voxelize_fuse(fm_ctx *ctx, const fm_pixel_map *in, const fm_sim3 *pose,
                           const fm_fusion_params *params, const float *accum, fm_surfel_buffer out,
                           int32_t *count, void *workspace, size_t ws_bytes, void *stream);

/* Workspace bytes fm_voxelize_fuse_batch needs for the n_frames maps of the
 * HOST array maps (only their sizes are read); 0 for n_frames < 1. */
size_t fm_fusion_batch_workspace_size(const fm_pixel_map *maps, int32_t n_frames);

/* fm_voxelize_fuse over several keyframes' maps in one set of launches (a
 * backlog of keyframes, or the frames of one fusion step).  maps, poses:
 * HOST arrays [n_frames]; accums: HOST array [n_frames] of DEVICE gate maps
 * (an entry may be NULL: no gate for that frame) or NULL (no gates).  The
 * survivors of frame 0, then frame 1, ... are written to out, each frame's
 * in fm_voxelize_fuse's order, so the result is the concatenation of
 * per-frame calls.  offsets: DEVICE int32 [n_frames + 1]; offsets[f] is the
 * position of frame f's first survivor and offsets[n_frames] the total,
 * reported even when it exceeds out.capacity (primitives beyond it are not
 * written).  Enqueued on stream; no allocation, no synchronisation;
 * graph-capturable (the per-frame descriptors travel as kernel arguments).
 * Errors: those of fm_voxelize_fuse for any frame, FM_ERR_INVALID_ARG for
 * n_frames < 1, NULL arrays or offsets, or a total pixel count of 2^31 or
 * more; FM_ERR_WORKSPACE when ws_bytes is below
 * fm_fusion_batch_workspace_size. */
fm_status fm_voxelize_fuse_batch(fm_ctx *ctx, const fm_pixel_map *maps, const fm_sim3 *poses, int32_t n_frames,
                                 const fm_fusion_params *params, const float *const *accums,
                                 fm_surfel_buffer out, int32_t *offsets, void *workspace, size_t ws_bytes,
                                 void *stream);

/* ---- map fusion: pruning the global map ---------------------------------
 *
 * Before new primitives join, the backend renders the global map from the
 * new keyframe's pose and removes the primitives that contribute to pixels
 * with a high RGB or depth reconstruction error (Sec. 3.3, "Map Fusion").
 * fm_prune_scores renders the batch (outputs as fm_forward writes them),
 * flags the high-error pixels -- (|I_r - I*_r| + |I_g - I*_g|) + |I_b - I*_b|,
 * divided by 3, above tau_rgb, or with a depth target |D - D*| above
 * tau_depth, each step in float32 -- and gives every surfel its score: the
 * sum over the flagged pixels of all views of its compositing weight
 * alpha_i T_i (its share in Eq. 1), summed in float32 in no fixed order.
 * fm_prune_compact then removes the surfels whose score exceeds a cut. */
typedef struct {
    const float *target_rgb;    /* DEVICE [3][P] observed image (unused with mask_in)         */
    const float *target_depth;  /* DEVICE [P] observed depth, or NULL: no depth criterion     */
    const uint8_t *mask_in;     /* DEVICE [P] or NULL: flag these pixels (non-zero) instead   */
    uint8_t *mask_out;          /* DEVICE [P] or NULL: receives the flags used (0/1)          */
    float tau_rgb;              /* mean absolute RGB error above which a pixel is flagged     */
    float tau_depth;            /* absolute depth error above which a pixel is flagged        */
} fm_prune_spec;

/* Scores of every surfel of every submap a view renders.  scores: HOST array
 * [n_submaps] of DEVICE float arrays [n of that submap], overwritten (an
 * entry may be NULL for a submap no view renders; such arrays are not
 * written).  Workspace, capacity and errors as fm_forward (query the pair
 * count with fm_query_status); the tile shape and order are the params'.
 * Enqueued on stream; no allocation, no synchronisation. */
fm_status fm_prune_scores(fm_ctx *ctx, const fm_batch *batch, const fm_raster_params *params,
                          const fm_prune_spec *spec, fm_outputs out, float *const *scores,
                          void *workspace, size_t ws_bytes, int64_t max_pairs, void *stream);

/* Workspace bytes fm_prune_compact needs for n surfels. */
size_t fm_prune_compact_workspace_size(int64_t n);

/* Removal: the surfels of `in` whose score (DEVICE [in->n]) is not above
 * tau_prune stay and are written, in their original order, to out; their
 * number goes to *count (DEVICE int32).  tau_prune = 0 removes every surfel
 * that contributes to a flagged pixel; a NaN score keeps its surfel.
 * Surfels beyond out.capacity are not written (*count still counts them).
 * Errors: FM_ERR_INVALID_ARG for NULL pointers, a negative size or
 * capacity, NULL output planes with capacity > 0, or a NaN tau_prune;
 * FM_ERR_WORKSPACE below fm_prune_compact_workspace_size.  Enqueued on
 * stream; no allocation, no synchronisation. */
fm_status fm_prune_compact(fm_ctx *ctx, const fm_surfels *in, const float *score, float tau_prune,
                           fm_surfel_buffer out, int32_t *count, void *workspace, size_t ws_bytes,
                           void *stream);

/* ---- loop correction of the map --------------------------------------------
 *
 * Primitives stay bound to the keyframe that created them (Sec. 3.3).  After
 * loop closure moves keyframe k from T_old to T_new, every primitive bound to
 * it is moved rigidly by Delta T_k = T_new T_old^-1, a similarity (s, q, t):
 * mu <- s R(q) mu + t, r <- q r (Hamilton product), scales <- s scales.
 * fm_warp_keyframes applies the moves in place to one surfel set.
 * mean [3][n], quat [4][n], scale [2][n]: DEVICE planes, updated in place.
 * keyframe: DEVICE int32 [n], the keyframe of each primitive; primitives
 * with an index outside [0, n_keyframes) are left alone.  deltas: DEVICE
 * [n_keyframes] Delta T per keyframe (the identity for keyframes that did
 * not move; q of any non-zero norm).  Enqueued on stream; no allocation;
 * graph-capturable.  Errors: FM_ERR_INVALID_ARG for a NULL context, NULL
 * planes with n > 0, a negative n or n_keyframes, or NULL deltas with
 * n_keyframes > 0; FM_ERR_HIP if the launch fails. */
fm_status fm_warp_keyframes(fm_ctx *ctx, float *mean, float *quat, float *scale, const int32_t *keyframe,
                            int64_t n, const fm_sim3 *deltas, int32_t n_keyframes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* FM2DGS_H */
