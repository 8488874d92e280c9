// fm_api.cpp -- the C ABI (include/fm2dgs.h): argument validation, workspace
// planning, and the launch sequences of forward, backward and the fused
// L1 forward+backward.  Every launch goes on the caller's stream; nothing here
// allocates device memory or synchronises on the hot path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "fm_internal.h"

using fm::Plan;
using fm::SubmapDesc;
using fm::ViewDesc;

struct fm_ctx {
    int device = 0;
    std::string name;
    int n_cu = 0;
    std::string last_error;
    struct Tuned {
        int tw, th, order, waves, depth;
    };
    std::map<std::string, Tuned> tuned;  // device arch + batch signature -> launch choice
    // device address of this device's copy of the library's static scratch
    // array (fm_fwd_bwd_l1_noalloc), resolved once per device by fm_create
    void *scratch = nullptr;
    // optional phase timing (benchmarks): events recorded between phases
    bool timing = false;
    hipEvent_t ev[8] = {};
    int marks = 0;
    int ev_phase[8] = {};
};

// Workspace of fm_fwd_bwd_l1_noalloc: a file-scope device array, one copy per
// GPU the library runs on, held until the process ends.  Host code never
// passes the array's name to a kernel or a copy (on the host it is only a
// stand-in symbol); it uses the device address that hipGetSymbolAddress
// returns for the current device.
static __device__ __align__(256) unsigned char scratch[FM_NOALLOC_SCRATCH_BYTES];

namespace {

// One device address per device, resolved with that device current.
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};

hipError_t scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    if (!g_scratch_ptr[device]) {
        int prev = -1;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev != device) (void)hipSetDevice(prev);
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// Copies the pair count of the last binning and its overflow flag out of the
// status word (fm_fwd_bwd_l1_noalloc's pair_status).
__global__ void k_pair_status(const fm::Status *st, int64_t *out) {
    if (threadIdx.x == 0) {
        out[0] = (int64_t)st->required;
        out[1] = st->overflow ? 1 : 0;
    }
}

constexpr int kVersion = 10000;  // 1.0.0

fm_status fail(fm_ctx *ctx, fm_status s, const std::string &msg) {
    if (ctx) ctx->last_error = msg;
    return s;
}

fm_status hip_fail(fm_ctx *ctx, hipError_t e, const char *where) {
    return fail(ctx, FM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

std::string signature(const fm_batch *b) {
    std::ostringstream os;
    os << "v" << b->n_views;
    for (int v = 0; v < b->n_views; ++v) {
        const fm_view_shape &s = b->views[v];
        const int n = b->submaps[s.submap].n;
        // bucket surfel counts to powers of two so nearby maps share a choice
        int nb = 0;
        while ((1 << nb) < n && nb < 31) ++nb;
        os << "_" << s.width << "x" << s.height << "n" << nb;
    }
    return os.str();
}

// Autotune cache key: the device's architecture and the batch signature;
// deterministic sums change the cost of each shape, so they tune separately.
std::string tune_key(const fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm) {
    return ctx->name + "/" + signature(b) + (prm->deterministic == 1 ? "/det" : "");
}

struct Built {
    Plan plan;
    std::vector<ViewDesc> views;
    std::vector<SubmapDesc> subs;
    std::vector<int32_t> vlist;
};

// The launch a call uses: the params' explicit choices, else the autotuned
// ones for this batch (when they were tuned for the same tile shape), else
// the defaults (16x16, longest list first, one wave per tile, depth 64).
struct Launch {
    int tw, th, order, waves, depth;
};

bool split_possible(int tw, int th) { return (tw == 16 && th == 16) || (tw == 16 && th == 8) || (tw == 32 && th == 8); }

fm_status resolve_launch(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm, Launch &L) {
    L.tw = prm->tile_w;
    L.th = prm->tile_h;
    auto it = ctx->tuned.find(tune_key(ctx, b, prm));
    const bool hit = it != ctx->tuned.end();
    if (L.tw == 0 && L.th == 0) {
        L.tw = hit ? it->second.tw : 16;
        L.th = hit ? it->second.th : 16;
    }
    if (!fm::tile_shape_supported(L.tw, L.th))
        return fail(ctx, FM_ERR_UNSUPPORTED, "unsupported tile shape " + std::to_string(L.tw) + "x" +
                                                 std::to_string(L.th) + " (use 8x8, 16x8, 16x16, 32x8 or 32x32)");
    if (prm->tile_order < 0 || prm->tile_order > 2)
        return fail(ctx, FM_ERR_INVALID_ARG, "tile_order must be 0, 1 or 2");
    if (prm->tile_waves < 0 || prm->tile_waves > 2)
        return fail(ctx, FM_ERR_INVALID_ARG, "tile_waves must be 0, 1 or 2");
    if (prm->lds_depth != 0 && prm->lds_depth != 32 && prm->lds_depth != 64 && prm->lds_depth != 128)
        return fail(ctx, FM_ERR_INVALID_ARG, "lds_depth must be 0, 32, 64 or 128");
    const bool same = hit && it->second.tw == L.tw && it->second.th == L.th;
    L.order = prm->tile_order != 0 ? prm->tile_order : (same ? it->second.order : 1);
    L.waves = prm->tile_waves != 0 ? prm->tile_waves : (same ? it->second.waves : 1);
    L.depth = prm->lds_depth != 0 ? prm->lds_depth : (same ? it->second.depth : 64);
    if (prm->deterministic == 1) {
        if (prm->lds_depth != 0 && prm->lds_depth != 64)
            return fail(ctx, FM_ERR_INVALID_ARG, "deterministic sums run with lds_depth 64 (or 0)");
        L.depth = 64;
    }
    if (!split_possible(L.tw, L.th)) L.waves = 1;  // 8x8: one block; 32x32: always four quadrant waves
    return FM_OK;
}

fm_status build(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm, int64_t max_pairs,
                const fm_surfel_grads *grads, bool need_backward, Built &out) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (!b || !prm) return fail(ctx, FM_ERR_INVALID_ARG, "batch and params must not be NULL");
    if (b->n_views < 1 || b->n_submaps < 1 || !b->views || !b->submaps)
        return fail(ctx, FM_ERR_INVALID_ARG, "a batch needs >= 1 view, >= 1 submap and host arrays for both");
    if (!b->intr || !b->viewmat) return fail(ctx, FM_ERR_INVALID_ARG, "intr and viewmat must not be NULL");
    if (!(prm->alpha_min >= 1e-6f) || !(prm->alpha_max > prm->alpha_min) || !(prm->alpha_max <= 1.f))
        return fail(ctx, FM_ERR_INVALID_ARG, "need 1e-6 <= alpha_min < alpha_max <= 1");
    if (need_backward && !(prm->alpha_max < 1.f))
        return fail(ctx, FM_ERR_INVALID_ARG, "the backward needs alpha_max < 1");
    if (!(prm->t_min >= 1e-30f && prm->t_min < 1.f)) return fail(ctx, FM_ERR_INVALID_ARG, "need 1e-30 <= t_min < 1");
    if (!(prm->rho_max > 0.f && std::isfinite(prm->rho_max)))
        return fail(ctx, FM_ERR_INVALID_ARG, "need rho_max > 0");
    if (!(prm->near_plane > 0.f && std::isfinite(prm->near_plane)))
        return fail(ctx, FM_ERR_INVALID_ARG, "need near_plane > 0");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(prm->bg[k])) return fail(ctx, FM_ERR_INVALID_ARG, "background must be finite");
    if (max_pairs < 1 || max_pairs > (int64_t)0x7FFFFFFF)
        return fail(ctx, FM_ERR_INVALID_ARG, "max_pairs must be in [1, 2^31-1]");
    Launch L;
    fm_status s = resolve_launch(ctx, b, prm, L);
    if (s != FM_OK) return s;
    const int tw = L.tw, th = L.th;

    Plan &p = out.plan;
    p = Plan();
    p.lpt = L.order == 1;
    p.split = L.waves == 2;
    p.depth = L.depth;
    p.V = b->n_views;
    p.S = b->n_submaps;
    p.tile_w = tw;
    p.tile_h = th;
    p.cap = max_pairs;
    if ((prm->deterministic != 0 && prm->deterministic != 1) || (prm->overwrite != 0 && prm->overwrite != 1))
        return fail(ctx, FM_ERR_INVALID_ARG, "deterministic and overwrite must be 0 or 1");
    p.det = prm->deterministic == 1;
    p.overwrite = prm->overwrite == 1;
    p.nq = (tw == 32 && th == 32) ? 4 : (p.split ? (tw / 8) * (th / 8) : 1);
    for (int i = 0; i < p.S; ++i) {
        const fm_surfels &sm = b->submaps[i];
        if (sm.n < 0 || sm.n > (1 << 28))
            return fail(ctx, FM_ERR_INVALID_ARG, "submap " + std::to_string(i) + ": n out of range");
        if (sm.n > 0 && (!sm.mean || !sm.quat || !sm.scale || !sm.opacity || !sm.color))
            return fail(ctx, FM_ERR_INVALID_ARG, "submap " + std::to_string(i) + ": NULL surfel plane");
    }
    out.views.resize(p.V);
    int64_t E = 0, T = 0, NPX = 0;
    for (int v = 0; v < p.V; ++v) {
        const fm_view_shape &vs = b->views[v];
        if (vs.width < 1 || vs.height < 1 || vs.width > 16384 || vs.height > 16384)
            return fail(ctx, FM_ERR_INVALID_ARG, "view " + std::to_string(v) + ": size out of [1, 16384]");
        if (vs.submap < 0 || vs.submap >= p.S)
            return fail(ctx, FM_ERR_INVALID_ARG, "view " + std::to_string(v) + ": submap index out of range");
        const fm_surfels &sm = b->submaps[vs.submap];
        ViewDesc &d = out.views[v];
        memset(&d, 0, sizeof(d));
        d.mean = sm.mean; d.quat = sm.quat; d.scale = sm.scale; d.opacity = sm.opacity; d.color = sm.color;
        d.n = sm.n;
        d.submap = vs.submap;
        d.entry_base = (int32_t)E;
        d.width = vs.width;
        d.height = vs.height;
        d.tiles_x = (vs.width + tw - 1) / tw;
        d.tiles_y = (vs.height + th - 1) / th;
        d.tile_base = (int32_t)T;
        d.pixel_offset = NPX;
        E += (int64_t)align_up((size_t)sm.n, fm::kEntryAlign);
        T += (int64_t)d.tiles_x * d.tiles_y;
        NPX += (int64_t)vs.width * vs.height;
        if (E > (int64_t)fm::kEntryMask || T > ((int64_t)1 << 31) || NPX > ((int64_t)1 << 31))
            return fail(ctx, FM_ERR_INVALID_ARG,
                        "batch too large (entries exceed 2^28, or tiles or pixels exceed 2^31)");
    }
    p.E = E;
    p.T = T;
    p.NPX = NPX;
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) < T) ++bits;
    p.tile_bits = bits;
    p.pair_passes = (bits + fm::kRadixBits - 1) / fm::kRadixBits;
    p.pairs_in_alt = (p.pair_passes & 1) != 0;
    auto grid_for = [](int64_t n) { return (int)std::max<int64_t>(1, (n + fm::kSortTile - 1) / fm::kSortTile); };
    p.sortG_e = grid_for(E);
    p.sortG_p = grid_for(max_pairs);
    p.scan_blocks = (int)std::max<int64_t>(1, (E + fm::kScanChunk - 1) / fm::kScanChunk);
    p.emit_blocks = std::min(p.sortG_p, fm::kMaxEmitGrid);  // a block emits one sort tile at a time

    // submaps in index order, each with the list of its views
    out.subs.resize(p.S);
    out.vlist.clear();
    int blocks = 0, max_blocks = 1, proj_blocks = 0;
    for (int sidx = 0; sidx < p.S; ++sidx) {
        const fm_surfels &sm = b->submaps[sidx];
        SubmapDesc &d = out.subs[sidx];
        memset(&d, 0, sizeof(d));
        d.mean = sm.mean; d.quat = sm.quat; d.scale = sm.scale; d.opacity = sm.opacity; d.color = sm.color;
        if (grads) {
            d.g_mean = grads[sidx].mean; d.g_quat = grads[sidx].quat; d.g_scale = grads[sidx].scale;
            d.g_opacity = grads[sidx].opacity; d.g_color = grads[sidx].color;
        }
        d.n = sm.n;
        d.view_begin = (int32_t)out.vlist.size();
        for (int v = 0; v < p.V; ++v)
            if (b->views[v].submap == sidx) out.vlist.push_back(v);
        d.view_count = (int32_t)out.vlist.size() - d.view_begin;
        d.block_base = blocks;
        const int nb = d.view_count > 0 ? (sm.n + 255) / 256 : 0;
        blocks += nb;
        d.proj_block_base = proj_blocks;
        proj_blocks += nb * ((d.view_count + fm::kProjViewsPerThread - 1) / fm::kProjViewsPerThread);
        max_blocks = std::max(max_blocks, (sm.n + 255) / 256);
    }
    p.a7_blocks = blocks;
    p.proj_blocks = proj_blocks;
    p.a7_max_blocks = max_blocks;

    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + std::max<size_t>(bytes, 1), 256);
        return at;
    };
    p.o_views = take(sizeof(ViewDesc) * p.V);
    p.o_subs = take(sizeof(SubmapDesc) * p.S);
    p.o_vlist = take(4 * (size_t)p.V);
    p.o_status = take(sizeof(fm::Status));
    p.o_rec = take(sizeof(fm::Rec) * (size_t)E);
    p.o_key = take(4 * (size_t)E);
    p.o_cnt = take(4 * (size_t)E);
    p.o_cnt2 = take(4 * (size_t)E);  // tile counts riding along the depth sort
    p.o_cnt3 = take(4 * (size_t)E);
    p.o_key2 = take(4 * (size_t)E);
    p.o_val = take(4 * (size_t)E);
    p.o_val2 = take(4 * (size_t)E);
    p.o_scan = take(4 * align_up(p.scan_blocks, 64));
    p.o_pkey = take(4 * (size_t)max_pairs);
    p.o_pval = take(4 * (size_t)max_pairs);
    p.o_pkey2 = take(4 * (size_t)max_pairs);
    p.o_pval2 = take(4 * (size_t)max_pairs);
    p.o_hist = take(4 * (size_t)fm::kRadix * std::max(p.sortG_e, p.sortG_p));
    p.o_tstart = take(4 * (size_t)T);
    p.o_tend = take(4 * (size_t)T);
    p.o_torder = take(4 * (size_t)T);  // blend order: tile ids, longest list first
    p.o_tbucket = take(4 * 2 * (size_t)fm::kRadix);  // its cost-bucket counts and cursors
    p.o_tfinal = take(4 * (size_t)NPX);
    p.o_nlast = take(4 * (size_t)NPX);
    p.o_ncount = take(4 * (size_t)NPX);
    p.o_grad = take(4 * fm::kGradStride * (size_t)E);
    p.o_ell = take(sizeof(fm::Ell) * (size_t)E);
    p.o_emeta = take(4 * (size_t)E);  // per entry: pixel-frame shift and normal flip (backward projection)
    p.o_pose = take(4 * 48 * (size_t)p.V * p.a7_max_blocks);  // 12 floats per (view, wave)
    p.o_loss = take(4 * (size_t)T * 16);
    p.o_tot = take(4 * (size_t)fm::kRadix * fm::kMaxPasses);
    p.o_chunk = take(4 * (size_t)((max_pairs + fm::kEmitChunk - 1) / fm::kEmitChunk + 1));
    if (p.det) {  // per pair: its value, and one partial gradient slot per wave of the tile
        p.o_meta = take(4 * (size_t)max_pairs);
        p.o_part = take(4 * (size_t)fm::kGradStride * p.nq * (size_t)max_pairs);
        p.o_pflag = take(align_up((size_t)p.nq * (size_t)max_pairs, 16));  // one byte per (pair, wave)
    }
    p.bytes = o;
    return FM_OK;
}

fm::KParams kparams(const fm_raster_params *prm, const Plan &p) {
    fm::KParams k;
    k.alpha_min = prm->alpha_min;
    k.alpha_max = prm->alpha_max;
    k.t_min = prm->t_min;
    k.rho_max = prm->rho_max;
    k.near_plane = prm->near_plane;
    k.bg[0] = prm->bg[0]; k.bg[1] = prm->bg[1]; k.bg[2] = prm->bg[2];
    k.tile_w = p.tile_w;
    k.tile_h = p.tile_h;
    k.gstride = fm::kGradSlot;
    k.pair_cap = (uint32_t)p.cap;
    return k;
}

fm_status check_ws(fm_ctx *ctx, const Plan &p, const void *ws, size_t ws_bytes) {
    if (!ws) return fail(ctx, FM_ERR_INVALID_ARG, "workspace must not be NULL");
    if (ws_bytes < p.bytes)
        return fail(ctx, FM_ERR_WORKSPACE, "workspace has " + std::to_string(ws_bytes) + " bytes, needs " +
                                               std::to_string(p.bytes));
    return FM_OK;
}

fm_status check_out(fm_ctx *ctx, const fm_outputs &o) {
    if (!o.rgb || !o.depth || !o.normal || !o.alpha)
        return fail(ctx, FM_ERR_INVALID_ARG, "every output plane must be non-NULL");
    return FM_OK;
}

fm_status use_device(fm_ctx *ctx) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipGetDevice");
    if (cur != ctx->device) {
        e = hipSetDevice(ctx->device);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
    }
    return FM_OK;
}

// Phase marks: phase ids as documented for fm_phase_times.
enum { PH_PRE = 0, PH_BIN = 1, PH_ZERO = 2, PH_BLEND = 3, PH_LOSS = 4, PH_BWDPROJ = 5, PH_N = 6 };

void mark_begin(fm_ctx *ctx, hipStream_t st) {
    ctx->marks = 0;
    if (!ctx->timing) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    if (hipEventRecord(ctx->ev[0], st) == hipSuccess) ctx->marks = 1;
}
void mark(fm_ctx *ctx, hipStream_t st, int phase) {
    if (!ctx->timing || ctx->marks == 0 || ctx->marks >= 8) return;
    if (hipEventRecord(ctx->ev[ctx->marks], st) == hipSuccess) ctx->ev_phase[ctx->marks++] = phase;
}

#define FM_TRY_HIP(expr, where)                      \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return hip_fail(ctx, _e, where); \
    } while (0)

// roctx ranges over a call and its phases (host-side spans of the enqueueing,
// shown by rocprofv3 --marker-trace next to the kernels they launch).
struct Ranges {
    int depth = 0;
    explicit Ranges(const char *call) {
        roctxRangePushA(call);
        depth = 1;
    }
    void phase(const char *name) {
        if (depth == 2) roctxRangePop();
        roctxRangePushA(name);
        depth = 2;
    }
    ~Ranges() {
        while (depth-- > 0) roctxRangePop();
    }
};

fm_status run_forward(fm_ctx *ctx, Built &bt, const fm_raster_params *prm, const fm_batch *b, void *ws,
                      const fm_outputs &out, hipStream_t st) {
    const fm::KParams kp = kparams(prm, bt.plan);
    Ranges rg("fm2dgs/forward");
    mark_begin(ctx, st);
    rg.phase("fm2dgs/projection");
    FM_TRY_HIP(fm::launch_setup(bt.plan, ws, bt.views.data(), bt.subs.data(), bt.vlist.data(), true, st), "setup");
    FM_TRY_HIP(fm::launch_preprocess(bt.plan, ws, kp, b->intr, b->viewmat, false, st), "preprocess");
    mark(ctx, st, PH_PRE);
    rg.phase("fm2dgs/binning");
    FM_TRY_HIP(fm::launch_binning(bt.plan, ws, st), "binning");
    mark(ctx, st, PH_BIN);
    rg.phase("fm2dgs/blend");
    FM_TRY_HIP(fm::launch_render_fwd(bt.plan, ws, kp, out, st), "render_fwd");
    mark(ctx, st, PH_BLEND);
    return FM_OK;
}

fm_status run_fused(fm_ctx *ctx, Built &bt, const fm_raster_params *prm, const fm_batch *b, void *ws,
                    const fm_l1_loss *ls, const fm_outputs &out, float *loss, float *dL_dviewmat,
                    hipStream_t st) {
    const fm::KParams kp = kparams(prm, bt.plan);
    fm::LossArgs la;
    la.target_rgb = ls->target_rgb;
    la.target_depth = ls->target_depth;
    la.mask = ls->mask;
    la.w_rgb = ls->w_rgb;
    la.w_depth = ls->w_depth;
    Ranges rg("fm2dgs/fwd_bwd_l1");
    mark_begin(ctx, st);
    rg.phase("fm2dgs/projection");
    FM_TRY_HIP(fm::launch_setup(bt.plan, ws, bt.views.data(), bt.subs.data(), bt.vlist.data(), true, st), "setup");
    // the slots are cleared for the blend's atomics; deterministic sums store
    // every slot the backward projection reads (those of visible entries)
    FM_TRY_HIP(fm::launch_preprocess(bt.plan, ws, kp, b->intr, b->viewmat, !bt.plan.det, st), "preprocess");
    mark(ctx, st, PH_PRE);
    rg.phase("fm2dgs/binning");
    FM_TRY_HIP(fm::launch_binning(bt.plan, ws, st), "binning");
    if (bt.plan.det) FM_TRY_HIP(fm::launch_det_clear(bt.plan, ws, kp.gstride, st), "det_clear");
    mark(ctx, st, PH_BIN);
    rg.phase("fm2dgs/blend");
    FM_TRY_HIP(fm::launch_render_fused(bt.plan, ws, kp, la, out, st), "render_fused");
    if (bt.plan.det) FM_TRY_HIP(fm::launch_det_reduce(bt.plan, ws, kp.gstride, st), "det_reduce");
    mark(ctx, st, PH_BLEND);
    rg.phase("fm2dgs/loss_reduce");
    FM_TRY_HIP(fm::launch_loss_reduce(bt.plan, ws, loss, st), "loss_reduce");
    mark(ctx, st, PH_LOSS);
    rg.phase("fm2dgs/backward_projection");
    FM_TRY_HIP(fm::launch_preprocess_bwd(bt.plan, ws, kp.gstride, b->intr, b->viewmat, dL_dviewmat, st),
               "preprocess_bwd");
    mark(ctx, st, PH_BWDPROJ);
    return FM_OK;
}

fm_status check_loss(fm_ctx *ctx, const fm_l1_loss *ls) {
    if (!ls) return fail(ctx, FM_ERR_INVALID_ARG, "loss spec must not be NULL");
    if (!ls->target_rgb) return fail(ctx, FM_ERR_INVALID_ARG, "target_rgb must not be NULL");
    if (ls->w_depth != 0.f && !ls->target_depth)
        return fail(ctx, FM_ERR_INVALID_ARG, "target_depth is required when w_depth != 0");
    if (!std::isfinite(ls->w_rgb) || !std::isfinite(ls->w_depth))
        return fail(ctx, FM_ERR_INVALID_ARG, "loss weights must be finite");
    return FM_OK;
}

// --- tiny JSON cache: {"arch/signature": [tw, th, tile order, waves, lds depth], ...} --
void load_cache(fm_ctx *ctx, const char *path) {
    std::ifstream f(path);
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t pos = 0;
    const std::string dev = "\"device\": \"";
    while (true) {
        size_t q0 = s.find('"', pos);
        if (q0 == std::string::npos) break;
        size_t q1 = s.find('"', q0 + 1);
        if (q1 == std::string::npos) break;
        const std::string key = s.substr(q0 + 1, q1 - q0 - 1);
        size_t lb = s.find('[', q1);
        size_t rb = s.find(']', q1);
        size_t nextq = s.find('"', q1 + 1);
        if (lb == std::string::npos || rb == std::string::npos || (nextq != std::string::npos && nextq < lb)) {
            pos = q1 + 1;
            continue;
        }
        int tw = 0, th = 0, order = 1, waves = 1, depth = 64;
        const int got = sscanf(s.c_str() + lb, "[%d, %d, %d, %d, %d]", &tw, &th, &order, &waves, &depth);
        if (got >= 2 && fm::tile_shape_supported(tw, th))
            ctx->tuned[key] = {tw, th, (got >= 3 && (order == 1 || order == 2)) ? order : 1,
                               (got >= 4 && waves == 2) ? 2 : 1,
                               (got >= 5 && (depth == 32 || depth == 128)) ? depth : 64};
        pos = rb + 1;
    }
}

void save_cache(fm_ctx *ctx, const char *path) {
    std::ofstream f(path);
    if (!f) return;
    f << "{\n";
    size_t k = 0;
    for (auto &kv : ctx->tuned) {
        f << "  \"" << kv.first << "\": [" << kv.second.tw << ", " << kv.second.th << ", " << kv.second.order << ", "
          << kv.second.waves << ", " << kv.second.depth << "]";
        f << (++k < ctx->tuned.size() ? ",\n" : "\n");
    }
    f << "}\n";
}

}  // namespace

extern "C" {

fm_status fm_create(fm_ctx **out, int device) {
    if (!out) return FM_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return FM_ERR_INVALID_ARG;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return FM_ERR_HIP;
    void *scratch_ptr = nullptr;
    if (scratch_address(device, &scratch_ptr) != hipSuccess) return FM_ERR_HIP;
    fm_ctx *c = new fm_ctx();
    c->device = device;
    c->name = prop.gcnArchName;
    c->n_cu = prop.multiProcessorCount;
    c->scratch = scratch_ptr;
    *out = c;
    return FM_OK;
}

void fm_destroy(fm_ctx *ctx) {
    if (!ctx) return;
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

fm_status fm_set_timing(fm_ctx *ctx, int enable) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (enable && !ctx->ev[0]) {
        fm_status s = use_device(ctx);
        if (s != FM_OK) return s;
        for (auto &e : ctx->ev) FM_TRY_HIP(hipEventCreate(&e), "hipEventCreate");
    }
    ctx->timing = enable != 0;
    ctx->marks = 0;
    return FM_OK;
}

fm_status fm_phase_times(fm_ctx *ctx, float *ms, int n) {
    if (!ctx || !ms || n < 6) return FM_ERR_INVALID_ARG;
    for (int k = 0; k < n; ++k) ms[k] = 0.f;
    if (ctx->marks < 2) return fail(ctx, FM_ERR_INVALID_ARG, "no timed call recorded (timing off or captured)");
    FM_TRY_HIP(hipEventSynchronize(ctx->ev[ctx->marks - 1]), "hipEventSynchronize");
    for (int k = 1; k < ctx->marks; ++k) {
        float t = 0.f;
        FM_TRY_HIP(hipEventElapsedTime(&t, ctx->ev[k - 1], ctx->ev[k]), "hipEventElapsedTime");
        ms[ctx->ev_phase[k]] += t;
    }
    return FM_OK;
}

fm_status fm_debug_counts(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm, const void *ws,
                          int64_t max_pairs, int64_t *n_visible, int64_t *n_kept) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    Built bt;
    fm_status s = build(ctx, b, prm, max_pairs, nullptr, false, bt);
    if (s != FM_OK) return s;
    if (!ws) return fail(ctx, FM_ERR_INVALID_ARG, "workspace must not be NULL");
    s = use_device(ctx);
    if (s != FM_OK) return s;
    fm::Status st;
    FM_TRY_HIP(hipMemcpy(&st, static_cast<const char *>(ws) + bt.plan.o_status, sizeof(st), hipMemcpyDeviceToHost),
               "hipMemcpy(status)");
    if (n_visible) *n_visible = st.n_vis;
    if (n_kept) *n_kept = st.n_kept;
    return FM_OK;
}

fm_status fm_bench_lds(fm_ctx *ctx, int32_t mode, int32_t blocks, int32_t iters, float *sink, double *lane_bytes,
                       void *stream) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if ((mode != 0 && mode != 1) || blocks < 1 || iters < 1 || !sink)
        return fail(ctx, FM_ERR_INVALID_ARG, "fm_bench_lds: mode 0 or 1, blocks >= 1, iters >= 1, sink not NULL");
    fm_status s = use_device(ctx);
    if (s != FM_OK) return s;
    FM_TRY_HIP(fm::launch_lds_probe(mode, blocks, iters, sink, (hipStream_t)stream), "lds_probe");
    if (lane_bytes) *lane_bytes = (double)fm::lds_probe_bytes(blocks, iters);
    return FM_OK;
}

fm_status fm_debug_pixel_state(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm, const void *ws,
                               int64_t max_pairs, float *t_final, uint32_t *n_contrib, int64_t npx) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    Built bt;
    fm_status s = build(ctx, b, prm, max_pairs, nullptr, false, bt);
    if (s != FM_OK) return s;
    if (!ws) return fail(ctx, FM_ERR_INVALID_ARG, "workspace must not be NULL");
    if (npx < bt.plan.NPX) return fail(ctx, FM_ERR_INVALID_ARG, "pixel buffers smaller than the batch");
    s = use_device(ctx);
    if (s != FM_OK) return s;
    const char *w = static_cast<const char *>(ws);
    if (t_final)
        FM_TRY_HIP(hipMemcpy(t_final, w + bt.plan.o_tfinal, 4 * bt.plan.NPX, hipMemcpyDeviceToHost), "hipMemcpy");
    if (n_contrib)
        FM_TRY_HIP(hipMemcpy(n_contrib, w + bt.plan.o_ncount, 4 * bt.plan.NPX, hipMemcpyDeviceToHost), "hipMemcpy");
    return FM_OK;
}

const char *fm_status_string(fm_status s) {
    switch (s) {
        case FM_OK: return "ok";
        case FM_ERR_INVALID_ARG: return "invalid argument";
        case FM_ERR_CAPACITY: return "pair capacity exceeded";
        case FM_ERR_HIP: return "HIP runtime error";
        case FM_ERR_UNSUPPORTED: return "unsupported configuration";
        case FM_ERR_WORKSPACE: return "workspace too small";
        default: return "unknown status";
    }
}

const char *fm_last_error(const fm_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "no context"; }

int fm_version(void) { return kVersion; }

void fm_default_params(fm_raster_params *p) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->alpha_min = 1.0f / 255.0f;
    p->alpha_max = 0.99f;
    p->t_min = 1e-4f;
    p->rho_max = 3.0f;
    p->near_plane = 0.2f;
    p->tile_w = 16;
    p->tile_h = 16;
}

fm_status fm_workspace_size(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm, int64_t max_pairs,
                            size_t *bytes) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (!bytes) return fail(ctx, FM_ERR_INVALID_ARG, "bytes must not be NULL");
    Built bt;
    fm_status s = build(ctx, b, prm, max_pairs, nullptr, false, bt);
    if (s != FM_OK) return s;
    *bytes = bt.plan.bytes;
    return FM_OK;
}

fm_status fm_tile_count(const fm_batch *b, const fm_raster_params *prm, int64_t *n_tiles) {
    if (!b || !prm || !n_tiles || !b->views || b->n_views < 1) return FM_ERR_INVALID_ARG;
    if (!fm::tile_shape_supported(prm->tile_w, prm->tile_h)) return FM_ERR_UNSUPPORTED;
    int64_t T = 0;
    for (int v = 0; v < b->n_views; ++v)
        T += (int64_t)((b->views[v].width + prm->tile_w - 1) / prm->tile_w) *
             ((b->views[v].height + prm->tile_h - 1) / prm->tile_h);
    *n_tiles = T;
    return FM_OK;
}

fm_status fm_forward(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm, fm_outputs out, void *ws,
                     size_t ws_bytes, int64_t max_pairs, void *stream) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    Built bt;
    fm_status s = build(ctx, b, prm, max_pairs, nullptr, false, bt);
    if (s == FM_OK) s = check_ws(ctx, bt.plan, ws, ws_bytes);
    if (s == FM_OK) s = check_out(ctx, out);
    if (s == FM_OK) s = use_device(ctx);
    if (s != FM_OK) return s;
    return run_forward(ctx, bt, prm, b, ws, out, (hipStream_t)stream);
}

fm_status fm_backward(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm, fm_outputs out,
                      fm_grad_outputs g, void *ws, size_t ws_bytes, int64_t max_pairs,
                      const fm_surfel_grads *grads, float *dL_dviewmat, void *stream) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (!grads) return fail(ctx, FM_ERR_INVALID_ARG, "grads must not be NULL (one entry per submap)");
    Built bt;
    fm_status s = build(ctx, b, prm, max_pairs, grads, true, bt);
    if (s == FM_OK) s = check_ws(ctx, bt.plan, ws, ws_bytes);
    if (s == FM_OK) s = check_out(ctx, out);
    if (s == FM_OK) s = use_device(ctx);
    if (s != FM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    fm::KParams kp = kparams(prm, bt.plan);
    if (g.normal) kp.gstride = fm::kGradStride;  // room for the normal's gradient
    Ranges rg("fm2dgs/backward");
    mark_begin(ctx, st);
    rg.phase("fm2dgs/zero_grad");
    FM_TRY_HIP(fm::launch_setup(bt.plan, ws, bt.views.data(), bt.subs.data(), bt.vlist.data(), false, st), "setup");
    if (bt.plan.det) FM_TRY_HIP(fm::launch_det_clear(bt.plan, ws, kp.gstride, st), "det_clear");
    else FM_TRY_HIP(fm::launch_zero_grad(bt.plan, ws, kp.gstride, st), "zero_grad");
    mark(ctx, st, PH_ZERO);
    rg.phase("fm2dgs/blend");
    FM_TRY_HIP(fm::launch_render_bwd(bt.plan, ws, kp, out, g, st), "render_bwd");
    if (bt.plan.det) FM_TRY_HIP(fm::launch_det_reduce(bt.plan, ws, kp.gstride, st), "det_reduce");
    mark(ctx, st, PH_BLEND);
    rg.phase("fm2dgs/backward_projection");
    FM_TRY_HIP(fm::launch_preprocess_bwd(bt.plan, ws, kp.gstride, b->intr, b->viewmat, dL_dviewmat, st),
               "preprocess_bwd");
    mark(ctx, st, PH_BWDPROJ);
    return FM_OK;
}

fm_status fm_fwd_bwd_l1(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm, const fm_l1_loss *ls,
                        fm_outputs out, float *loss, const fm_surfel_grads *grads, float *dL_dviewmat, void *ws,
                        size_t ws_bytes, int64_t max_pairs, void *stream) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (!grads) return fail(ctx, FM_ERR_INVALID_ARG, "grads must not be NULL (one entry per submap)");
    Built bt;
    fm_status s = build(ctx, b, prm, max_pairs, grads, true, bt);
    if (s == FM_OK) s = check_ws(ctx, bt.plan, ws, ws_bytes);
    if (s == FM_OK) s = check_out(ctx, out);
    if (s == FM_OK) s = check_loss(ctx, ls);
    if (s == FM_OK) s = use_device(ctx);
    if (s != FM_OK) return s;
    return run_fused(ctx, bt, prm, b, ws, ls, out, loss, dL_dviewmat, (hipStream_t)stream);
}

fm_status fm_fwd_bwd_l1_noalloc(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm,
                                const fm_l1_loss *ls, fm_outputs out, float *loss, const fm_surfel_grads *grads,
                                float *dL_dviewmat, int64_t max_pairs, int64_t *pair_status, void *stream) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (!grads) return fail(ctx, FM_ERR_INVALID_ARG, "grads must not be NULL (one entry per submap)");
    if (!ctx->scratch) return fail(ctx, FM_ERR_HIP, "the static scratch array has no device address");
    Built bt;
    fm_status s = build(ctx, b, prm, max_pairs, grads, true, bt);
    if (s != FM_OK) return s;
    if (bt.plan.bytes > (size_t)FM_NOALLOC_SCRATCH_BYTES)
        return fail(ctx, FM_ERR_WORKSPACE,
                    "fm_fwd_bwd_l1_noalloc: the batch needs " + std::to_string(bt.plan.bytes) +
                        " bytes of workspace, the static scratch holds " +
                        std::to_string((size_t)FM_NOALLOC_SCRATCH_BYTES) + " (use fm_fwd_bwd_l1)");
    s = check_out(ctx, out);
    if (s == FM_OK) s = check_loss(ctx, ls);
    if (s == FM_OK) s = use_device(ctx);
    if (s != FM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    s = run_fused(ctx, bt, prm, b, ctx->scratch, ls, out, loss, dL_dviewmat, st);
    if (s != FM_OK || !pair_status) return s;
    hipLaunchKernelGGL(k_pair_status, dim3(1), dim3(64), 0, st, fm::at<fm::Status>(ctx->scratch, bt.plan.o_status),
                       pair_status);
    FM_TRY_HIP(hipGetLastError(), "pair_status");
    return FM_OK;
}

fm_status fm_prune_scores(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm, const fm_prune_spec *spec,
                          fm_outputs out, float *const *scores, void *ws, size_t ws_bytes, int64_t max_pairs,
                          void *stream) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (!spec || !scores) return fail(ctx, FM_ERR_INVALID_ARG, "fm_prune_scores: spec and scores must not be NULL");
    if (!spec->mask_in) {
        if (!spec->target_rgb)
            return fail(ctx, FM_ERR_INVALID_ARG, "fm_prune_scores: target_rgb is needed without mask_in");
        if (!std::isfinite(spec->tau_rgb) || (spec->target_depth && !std::isfinite(spec->tau_depth)))
            return fail(ctx, FM_ERR_INVALID_ARG, "fm_prune_scores: thresholds must be finite");
    }
    if (!b || b->n_submaps < 1) return fail(ctx, FM_ERR_INVALID_ARG, "batch must not be NULL");
    // the per-surfel reduction stores each submap's scores through the g_opacity slot
    std::vector<fm_surfel_grads> dst((size_t)b->n_submaps);
    for (int i = 0; i < b->n_submaps; ++i) {
        memset(&dst[i], 0, sizeof(dst[i]));
        dst[i].opacity = scores[i];
    }
    Built bt;
    fm_status s = build(ctx, b, prm, max_pairs, dst.data(), false, bt);
    if (s == FM_OK) s = check_ws(ctx, bt.plan, ws, ws_bytes);
    if (s == FM_OK) s = check_out(ctx, out);
    if (s == FM_OK) s = use_device(ctx);
    if (s != FM_OK) return s;
    for (int i = 0; i < b->n_submaps; ++i)
        if (!scores[i] && bt.subs[i].view_count > 0 && b->submaps[i].n > 0)
            return fail(ctx, FM_ERR_INVALID_ARG,
                        "fm_prune_scores: scores[" + std::to_string(i) + "] is NULL but a view renders submap");
    hipStream_t st = (hipStream_t)stream;
    fm::KParams kp = kparams(prm, bt.plan);
    fm::PruneArgs pa;
    pa.target_rgb = spec->target_rgb;
    pa.target_depth = spec->target_depth;
    pa.mask_in = spec->mask_in;
    pa.mask_out = spec->mask_out;
    pa.tau_rgb = spec->tau_rgb;
    pa.tau_depth = spec->tau_depth;
    Ranges rg("fm2dgs/prune_scores");
    mark_begin(ctx, st);
    rg.phase("fm2dgs/projection");
    FM_TRY_HIP(fm::launch_setup(bt.plan, ws, bt.views.data(), bt.subs.data(), bt.vlist.data(), true, st), "setup");
    // the projection clears the slots whose first float collects each entry's score
    FM_TRY_HIP(fm::launch_preprocess(bt.plan, ws, kp, b->intr, b->viewmat, true, st), "preprocess");
    mark(ctx, st, PH_PRE);
    rg.phase("fm2dgs/binning");
    FM_TRY_HIP(fm::launch_binning(bt.plan, ws, st), "binning");
    mark(ctx, st, PH_BIN);
    rg.phase("fm2dgs/blend");
    FM_TRY_HIP(fm::launch_render_prune(bt.plan, ws, kp, pa, out, st), "render_prune");
    mark(ctx, st, PH_BLEND);
    rg.phase("fm2dgs/score_reduce");
    FM_TRY_HIP(fm::launch_score_reduce(bt.plan, ws, kp.gstride, st), "score_reduce");
    mark(ctx, st, PH_BWDPROJ);
    return FM_OK;
}

size_t fm_prune_compact_workspace_size(int64_t n) { return n < 0 ? 0 : fm::prune_compact_workspace_bytes(n); }

fm_status fm_prune_compact(fm_ctx *ctx, const fm_surfels *in, const float *score, float tau_prune,
                           fm_surfel_buffer out, int32_t *count, void *ws, size_t ws_bytes, void *stream) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (!in || !count || !ws) return fail(ctx, FM_ERR_INVALID_ARG, "fm_prune_compact: NULL in, count or workspace");
    if (in->n < 0) return fail(ctx, FM_ERR_INVALID_ARG, "fm_prune_compact: negative n");
    if (in->n > 0 && (!score || !in->mean || !in->quat || !in->scale || !in->opacity || !in->color))
        return fail(ctx, FM_ERR_INVALID_ARG, "fm_prune_compact: NULL surfel plane or score");
    if (out.capacity < 0 ||
        (out.capacity > 0 && (!out.mean || !out.quat || !out.scale || !out.opacity || !out.color)))
        return fail(ctx, FM_ERR_INVALID_ARG, "fm_prune_compact: negative capacity or NULL output plane");
    if (std::isnan(tau_prune)) return fail(ctx, FM_ERR_INVALID_ARG, "fm_prune_compact: tau_prune is NaN");
    if (ws_bytes < fm::prune_compact_workspace_bytes(in->n))
        return fail(ctx, FM_ERR_WORKSPACE, "fm_prune_compact: workspace smaller than fm_prune_compact_workspace_size");
    fm_status s = use_device(ctx);
    if (s != FM_OK) return s;
    FM_TRY_HIP(fm::launch_prune_compact(*in, score, tau_prune, out, count, ws, (hipStream_t)stream), "prune_compact");
    return FM_OK;
}

fm_status fm_query_status(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm, const void *ws,
                          int64_t max_pairs, int64_t *n_pairs, int64_t *required) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    Built bt;
    fm_status s = build(ctx, b, prm, max_pairs, nullptr, false, bt);
    if (s != FM_OK) return s;
    if (!ws) return fail(ctx, FM_ERR_INVALID_ARG, "workspace must not be NULL");
    s = use_device(ctx);
    if (s != FM_OK) return s;
    fm::Status st;
    FM_TRY_HIP(hipMemcpy(&st, static_cast<const char *>(ws) + bt.plan.o_status, sizeof(st), hipMemcpyDeviceToHost),
               "hipMemcpy(status)");
    if (n_pairs) *n_pairs = st.n_pairs;
    if (required) *required = (int64_t)st.required;
    if (st.overflow) {
        ctx->last_error = "pair buffer overflow: " + std::to_string(st.required) + " pairs needed, capacity " +
                          std::to_string(max_pairs);
        return FM_ERR_CAPACITY;
    }
    return FM_OK;
}

fm_status fm_debug_pairs(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm, const void *ws,
                         int64_t max_pairs, uint32_t *tile, uint32_t *surfel, uint32_t *view, int64_t cap,
                         int64_t *n_pairs, uint32_t *tile_start, uint32_t *tile_end, int64_t n_tiles) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    Built bt;
    fm_status s = build(ctx, b, prm, max_pairs, nullptr, false, bt);
    if (s != FM_OK) return s;
    const Plan &p = bt.plan;
    if (!ws || !n_pairs) return fail(ctx, FM_ERR_INVALID_ARG, "workspace and n_pairs must not be NULL");
    s = use_device(ctx);
    if (s != FM_OK) return s;
    fm::Status st;
    const char *w = static_cast<const char *>(ws);
    FM_TRY_HIP(hipMemcpy(&st, w + p.o_status, sizeof(st), hipMemcpyDeviceToHost), "hipMemcpy(status)");
    *n_pairs = st.n_kept;
    const int64_t m = std::min<int64_t>(st.n_kept, cap);
    if (m > 0 && (tile || surfel || view)) {
        std::vector<uint32_t> k(m), e(m);
        FM_TRY_HIP(hipMemcpy(k.data(), w + (p.pairs_in_alt ? p.o_pkey2 : p.o_pkey), 4 * m, hipMemcpyDeviceToHost),
                   "hipMemcpy(pairs)");
        FM_TRY_HIP(hipMemcpy(e.data(), w + (p.pairs_in_alt ? p.o_pval2 : p.o_pval), 4 * m, hipMemcpyDeviceToHost),
                   "hipMemcpy(pairs)");
        if (p.det && st.n_pairs > 0) {  // the list holds emission indices
            std::vector<uint32_t> meta(st.n_pairs);
            FM_TRY_HIP(hipMemcpy(meta.data(), w + p.o_meta, 4 * (size_t)st.n_pairs, hipMemcpyDeviceToHost),
                       "hipMemcpy(pairs)");
            for (int64_t i = 0; i < m; ++i) e[i] = e[i] < st.n_pairs ? meta[e[i]] : 0u;
        }
        for (int64_t i = 0; i < m; ++i) {
            int lo = 0, hi = p.V - 1;
            while (lo < hi) {
                int mid = (lo + hi + 1) / 2;
                if ((uint32_t)bt.views[mid].entry_base <= (e[i] & fm::kEntryMask)) lo = mid; else hi = mid - 1;
            }
            if (tile) tile[i] = k[i];
            if (surfel) surfel[i] = (e[i] & fm::kEntryMask) - (uint32_t)bt.views[lo].entry_base;
            if (view) view[i] = (uint32_t)lo;
        }
    }
    if (tile_start && tile_end) {
        if (n_tiles < p.T) return fail(ctx, FM_ERR_INVALID_ARG, "tile range buffers too small");
        FM_TRY_HIP(hipMemcpy(tile_start, w + p.o_tstart, 4 * p.T, hipMemcpyDeviceToHost), "hipMemcpy(ranges)");
        FM_TRY_HIP(hipMemcpy(tile_end, w + p.o_tend, 4 * p.T, hipMemcpyDeviceToHost), "hipMemcpy(ranges)");
        for (int64_t t = 0; t < p.T; ++t)  // a tile without pairs is stored as ts > te
            if (tile_start[t] > tile_end[t]) tile_start[t] = tile_end[t] = 0u;
    }
    return FM_OK;
}

fm_status fm_autotune(fm_ctx *ctx, const fm_batch *b, const fm_raster_params *prm, const fm_l1_loss *ls,
                      fm_outputs out, float *loss, const fm_surfel_grads *grads, float *dL_dviewmat, void *ws,
                      size_t ws_bytes, int64_t max_pairs, const char *cache_path, fm_raster_params *chosen,
                      void *stream) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (!chosen || !prm || !b) return fail(ctx, FM_ERR_INVALID_ARG, "batch, params and chosen must not be NULL");
    if (cache_path) load_cache(ctx, cache_path);
    const std::string sig = tune_key(ctx, b, prm);
    *chosen = *prm;
    auto put = [&](const fm_ctx::Tuned &t) {
        chosen->tile_w = t.tw;
        chosen->tile_h = t.th;
        chosen->tile_order = t.order;
        chosen->tile_waves = t.waves;
        chosen->lds_depth = t.depth;
    };
    auto hit = ctx->tuned.find(sig);
    if (hit != ctx->tuned.end()) {
        put(hit->second);
        return FM_OK;
    }
    fm_status s = check_loss(ctx, ls);
    if (s == FM_OK) s = check_out(ctx, out);
    if (s == FM_OK) s = use_device(ctx);
    if (s != FM_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    // one event per call boundary: each call is timed on its own and a
    // candidate is scored by the median, so that one slow call (a clock
    // change, another process on the device) does not decide the choice
    constexpr int kMaxReps = 15;
    struct Events {  // destroyed on every return path
        hipEvent_t e[kMaxReps + 1] = {};
        ~Events() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev;
    for (hipEvent_t &x : ev.e) FM_TRY_HIP(hipEventCreate(&x), "hipEventCreate");
    // Times one candidate: a warm-up call and its pair status, then `reps`
    // calls (each call's status checked), each between two events; `ms` is
    // the median call.  A candidate that does not fit the workspace or the
    // pair capacity gets ms < 0 (skipped).
    auto time_one = [&](const fm_ctx::Tuned &t, int reps, float &ms) -> fm_status {
        fm_raster_params q = *prm;
        q.tile_w = t.tw;
        q.tile_h = t.th;
        q.tile_order = t.order;
        q.tile_waves = t.waves;
        q.lds_depth = t.depth;
        Built bt;
        fm_status r = build(ctx, b, &q, max_pairs, grads, true, bt);
        ms = -1.f;
        if (r != FM_OK || bt.plan.bytes > ws_bytes) return FM_OK;  // does not fit: skipped
        r = run_fused(ctx, bt, &q, b, ws, ls, out, loss, dL_dviewmat, st);
        if (r != FM_OK) return r;
        FM_TRY_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
        fm::Status stt;
        FM_TRY_HIP(hipMemcpy(&stt, static_cast<char *>(ws) + bt.plan.o_status, sizeof(stt), hipMemcpyDeviceToHost),
                   "hipMemcpy(status)");
        if (stt.overflow) return FM_OK;  // capacity too small for this shape: skipped
        reps = std::max(1, std::min(reps, kMaxReps));
        FM_TRY_HIP(hipEventRecord(ev.e[0], st), "hipEventRecord");
        for (int k = 0; k < reps; ++k) {
            r = run_fused(ctx, bt, &q, b, ws, ls, out, loss, dL_dviewmat, st);
            if (r != FM_OK) return r;
            FM_TRY_HIP(hipEventRecord(ev.e[k + 1], st), "hipEventRecord");
        }
        FM_TRY_HIP(hipEventSynchronize(ev.e[reps]), "hipEventSynchronize");
        float dt[kMaxReps];
        for (int k = 0; k < reps; ++k)
            FM_TRY_HIP(hipEventElapsedTime(&dt[k], ev.e[k], ev.e[k + 1]), "hipEventElapsedTime");
        std::sort(dt, dt + reps);
        ms = dt[reps / 2];
        return FM_OK;
    };
    // Stage 1: every tile shape with both tile orders and, where a tile holds
    // several 8x8 blocks, one wave per tile or per block, at LDS depth 64 and
    // a few calls each.  Stage 2: the default launch (16x16, longest list
    // first, one wave per tile, depth 64) and the three fastest of stage 1,
    // each at LDS depths 64, 32 and 128 (deterministic sums keep depth 64),
    // with more calls.  A candidate replaces the best so far only when its
    // median is more than 1% lower, so that timing noise does not move the
    // choice away from the default.
    const int shapes[5][2] = {{16, 16}, {8, 8}, {16, 8}, {32, 8}, {32, 32}};
    const fm_ctx::Tuned dflt = {16, 16, 1, 1, 64};
    std::vector<std::pair<float, fm_ctx::Tuned>> stage1;
    for (const auto &sh : shapes) {
        for (int waves = 1; waves <= (split_possible(sh[0], sh[1]) ? 2 : 1); ++waves) {
            for (int order = 1; order <= 2; ++order) {
                const fm_ctx::Tuned t = {sh[0], sh[1], order, waves, 64};
                float ms;
                s = time_one(t, 5, ms);
                if (s != FM_OK) return s;
                if (ms >= 0.f) stage1.push_back({ms, t});
            }
        }
    }
    if (stage1.empty()) return fail(ctx, FM_ERR_WORKSPACE, "no tile shape fits the workspace and capacity");
    std::stable_sort(stage1.begin(), stage1.end(),
                     [](const auto &x, const auto &y) { return x.first < y.first; });
    auto same = [](const fm_ctx::Tuned &x, const fm_ctx::Tuned &y) {
        return x.tw == y.tw && x.th == y.th && x.order == y.order && x.waves == y.waves && x.depth == y.depth;
    };
    std::vector<fm_ctx::Tuned> stage2;
    for (const auto &c : stage1)
        if (same(c.second, dflt)) stage2.push_back(dflt);  // only when it fits
    for (size_t i = 0; i < stage1.size() && i < 3; ++i)
        if (!same(stage1[i].second, dflt)) stage2.push_back(stage1[i].second);
    float best = 1e30f;
    fm_ctx::Tuned bt_best = stage1[0].second;
    for (const fm_ctx::Tuned &c : stage2) {
        for (int depth : {64, 32, 128}) {
            if (depth != 64 && prm->deterministic == 1) continue;
            fm_ctx::Tuned t = c;
            t.depth = depth;
            float ms;
            s = time_one(t, kMaxReps, ms);
            if (s != FM_OK) return s;
            if (ms >= 0.f && ms < 0.99f * best) {
                best = ms;
                bt_best = t;
            }
        }
    }
    ctx->tuned[sig] = bt_best;
    if (cache_path) save_cache(ctx, cache_path);
    put(bt_best);
    return FM_OK;
}

fm_status fm_adam_step(fm_ctx *ctx, const fm_adam_tensor *tensors, int32_t count, const fm_adam_config *config,
                       int32_t *step, void *stream) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (!config || !step || count < 0 || (count > 0 && !tensors))
        return fail(ctx, FM_ERR_INVALID_ARG, "fm_adam_step: NULL config/step/tensors or negative count");
    if (!(config->beta1 >= 0.f && config->beta1 < 1.f) || !(config->beta2 >= 0.f && config->beta2 < 1.f) ||
        !(config->eps > 0.f))
        return fail(ctx, FM_ERR_INVALID_ARG, "fm_adam_step: need 0 <= beta1, beta2 < 1 and eps > 0");
    for (int32_t k = 0; k < count; ++k) {
        const fm_adam_tensor &t = tensors[k];
        if (t.n < 0 || t.n >= ((int64_t)1 << 31) || (t.n > 0 && (!t.param || !t.grad || !t.m || !t.v)))
            return fail(ctx, FM_ERR_INVALID_ARG, "fm_adam_step: tensor " + std::to_string(k) +
                                                     " has a negative or too large size or a NULL buffer");
        if (!(t.lr > 0.f) || !std::isfinite(t.lr))
            return fail(ctx, FM_ERR_INVALID_ARG, "fm_adam_step: tensor " + std::to_string(k) + " needs lr > 0");
        if (t.kind != FM_PARAM_LINEAR && t.kind != FM_PARAM_LOG && t.kind != FM_PARAM_LOGIT)
            return fail(ctx, FM_ERR_INVALID_ARG, "fm_adam_step: tensor " + std::to_string(k) + " has an unknown kind");
    }
    fm_status s = use_device(ctx);
    if (s != FM_OK) return s;
    FM_TRY_HIP(fm::launch_adam(tensors, count, *config, step, (hipStream_t)stream), "adam");
    return FM_OK;
}

size_t fm_fusion_workspace_size(int32_t width, int32_t height) {
    if (width < 1 || height < 1) return 0;
    return fm::fusion_workspace_bytes(width, height);
}

}  // extern "C"

namespace {
// Checks of one frame of a fusion call; the message names the entry point.
fm_status check_frame(fm_ctx *ctx, const char *fn, const fm_pixel_map *in, const fm_sim3 *pose) {
    const std::string f = fn;
    if (!in || !pose) return fail(ctx, FM_ERR_INVALID_ARG, f + ": NULL map or pose");
    if (in->width < 1 || in->height < 1 || (int64_t)in->width * in->height >= ((int64_t)1 << 31))
        return fail(ctx, FM_ERR_INVALID_ARG, f + ": need width, height >= 1 and width*height < 2^31");
    if (!in->mean || !in->quat || !in->scale || !in->opacity || !in->color)
        return fail(ctx, FM_ERR_INVALID_ARG, f + ": NULL input plane");
    const double qq = (double)pose->q[0] * pose->q[0] + (double)pose->q[1] * pose->q[1] +
                      (double)pose->q[2] * pose->q[2] + (double)pose->q[3] * pose->q[3];
    if (!(pose->s > 0.f) || !std::isfinite(pose->s) || !(qq > 0.0) || !std::isfinite(qq) ||
        !std::isfinite(pose->t[0]) || !std::isfinite(pose->t[1]) || !std::isfinite(pose->t[2]))
        return fail(ctx, FM_ERR_INVALID_ARG, f + ": need s > 0 and a finite, non-zero pose");
    return FM_OK;
}
fm_status check_surfel_out(fm_ctx *ctx, const char *fn, const fm_surfel_buffer &out) {
    if (out.capacity < 0 ||
        (out.capacity > 0 && (!out.mean || !out.quat || !out.scale || !out.opacity || !out.color)))
        return fail(ctx, FM_ERR_INVALID_ARG, std::string(fn) + ": bad output buffer");
    return FM_OK;
}
}  // namespace

extern "C" {

fm_status fm_voxelize_fuse(fm_ctx *ctx, const fm_pixel_map *in, const fm_sim3 *pose,
                           const fm_fusion_params *params, const float *accum, fm_surfel_buffer out,
                           int32_t *count, void *workspace, size_t ws_bytes, void *stream) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (!params || !count || !workspace)
        return fail(ctx, FM_ERR_INVALID_ARG, "fm_voxelize_fuse: NULL params, count or workspace");
    fm_status s = check_frame(ctx, "fm_voxelize_fuse", in, pose);
    if (s != FM_OK) return s;
    s = check_surfel_out(ctx, "fm_voxelize_fuse", out);
    if (s != FM_OK) return s;
    if (ws_bytes < fm::fusion_workspace_bytes(in->width, in->height))
        return fail(ctx, FM_ERR_WORKSPACE, "fm_voxelize_fuse: workspace too small");
    s = use_device(ctx);
    if (s != FM_OK) return s;
    FM_TRY_HIP(fm::launch_fusion(*in, *pose, *params, accum, out, count, workspace, (hipStream_t)stream), "fusion");
    return FM_OK;
}

size_t fm_fusion_batch_workspace_size(const fm_pixel_map *maps, int32_t n_frames) {
    if (!maps || n_frames < 1) return 0;
    for (int32_t f = 0; f < n_frames; ++f)
        if (maps[f].width < 1 || maps[f].height < 1) return 0;
    return fm::fusion_batch_workspace_bytes(maps, n_frames);
}

fm_status fm_voxelize_fuse_batch(fm_ctx *ctx, const fm_pixel_map *maps, const fm_sim3 *poses, int32_t n_frames,
                                 const fm_fusion_params *params, const float *const *accums,
                                 fm_surfel_buffer out, int32_t *offsets, void *workspace, size_t ws_bytes,
                                 void *stream) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (n_frames < 1 || !maps || !poses || !params || !offsets || !workspace)
        return fail(ctx, FM_ERR_INVALID_ARG,
                    "fm_voxelize_fuse_batch: need n_frames >= 1 and non-NULL maps, poses, params, offsets, workspace");
    int64_t px = 0;
    for (int32_t f = 0; f < n_frames; ++f) {
        fm_status s = check_frame(ctx, "fm_voxelize_fuse_batch", maps + f, poses + f);
        if (s != FM_OK) return s;
        px += (int64_t)maps[f].width * maps[f].height;
    }
    if (px >= ((int64_t)1 << 31))
        return fail(ctx, FM_ERR_INVALID_ARG, "fm_voxelize_fuse_batch: the frames hold 2^31 pixels or more");
    fm_status s = check_surfel_out(ctx, "fm_voxelize_fuse_batch", out);
    if (s != FM_OK) return s;
    if (ws_bytes < fm::fusion_batch_workspace_bytes(maps, n_frames))
        return fail(ctx, FM_ERR_WORKSPACE, "fm_voxelize_fuse_batch: workspace too small");
    s = use_device(ctx);
    if (s != FM_OK) return s;
    FM_TRY_HIP(fm::launch_fusion_batch(maps, poses, n_frames, *params, accums, out, offsets, offsets + n_frames,
                                       workspace, (hipStream_t)stream),
               "fusion_batch");
    return FM_OK;
}

fm_status fm_warp_keyframes(fm_ctx *ctx, float *mean, float *quat, float *scale, const int32_t *keyframe,
                            int64_t n, const fm_sim3 *deltas, int32_t n_keyframes, void *stream) {
    if (!ctx) return FM_ERR_INVALID_ARG;
    if (n < 0 || n_keyframes < 0 || (n > 0 && (!mean || !quat || !scale || !keyframe)) ||
        (n_keyframes > 0 && !deltas))
        return fail(ctx, FM_ERR_INVALID_ARG, "fm_warp_keyframes: NULL buffer or negative size");
    fm_status s = use_device(ctx);
    if (s != FM_OK) return s;
    FM_TRY_HIP(fm::launch_warp(mean, quat, scale, keyframe, n, deltas, n_keyframes, (hipStream_t)stream), "warp");
    return FM_OK;
}

}  // extern "C"
