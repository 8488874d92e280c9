"""PyTorch-facing binding of the gfx950 surfel rasterizer.

PyTorch only provides device memory and the current stream; every step of
projection, binning, sorting, compositing and their adjoints runs in
libfm2dgs.so through the C ABI declared in include/fm2dgs.h.

    rast = Rasterizer()
    gs = GpuScene.from_scene(scenes.config1())
    out, ws = rast.forward(gs)
    rast.backward(gs, ws, out, dL_dout, grads, dL_dviewmat)

``render`` wraps the same calls in a torch.autograd.Function.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import native
from .native import (FmBatch, FmGradOutputs, FmL1Loss, FmOutputs, FmRasterParams, FmSurfelGrads, FmSurfels,
                     FmViewShape)

PLANES = ("mean", "quat", "scale", "opacity", "color")
CHANNELS = {"mean": 3, "quat": 4, "scale": 2, "opacity": 1, "color": 3}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class GpuScene:
    """Device tensors of a batch (surfel submaps, views, cameras, targets) and
    the C-ABI batch descriptor pointing at them."""

    def __init__(self, submaps, views, intr, viewmat, target_rgb=None, target_depth=None,
                 w_rgb=1.0, w_depth=0.0, name="scene"):
        self.submaps = submaps
        self.views = [tuple(int(x) for x in v) for v in views]
        self.intr = intr.contiguous()
        self.viewmat = viewmat.contiguous()
        self.target_rgb = target_rgb
        self.target_depth = target_depth
        self.w_rgb = float(w_rgb)
        self.w_depth = float(w_depth)
        self.name = name
        self.npx = sum(w * h for (w, h, _) in self.views)
        self.pixel_offsets = []
        off = 0
        for (w, h, _) in self.views:
            self.pixel_offsets.append(off)
            off += w * h
        self._batch = None

    @classmethod
    def from_scene(cls, scene, device="cuda"):
        subs = [{k: torch.from_numpy(sm[k]).to(device).contiguous() for k in PLANES} for sm in scene.submaps]
        f = lambda a: None if a is None else torch.from_numpy(a).to(device).contiguous()
        return cls(subs, scene.views, f(scene.intr), f(scene.viewmat), f(scene.target_rgb),
                   f(scene.target_depth), scene.w_rgb, scene.w_depth, scene.name)

    @property
    def n_views(self):
        return len(self.views)

    def batch(self):
        """FmBatch (cached; rebuilt if a tensor was replaced)."""
        key = tuple(t.data_ptr() for sm in self.submaps for t in sm.values()) + (
            self.intr.data_ptr(), self.viewmat.data_ptr())
        if self._batch is None or self._batch[0] != key:
            subs = (FmSurfels * len(self.submaps))()
            for i, sm in enumerate(self.submaps):
                subs[i].n = int(sm["opacity"].shape[-1])
                for k in PLANES:
                    assert sm[k].is_contiguous() and sm[k].dtype == torch.float32
                    assert sm[k].shape[-1] == subs[i].n and sm[k].numel() == CHANNELS[k] * subs[i].n
                    setattr(subs[i], k, sm[k].data_ptr())
            vs = (FmViewShape * len(self.views))()
            for i, (w, h, s) in enumerate(self.views):
                vs[i].width, vs[i].height, vs[i].submap = w, h, s
            b = FmBatch(len(self.submaps), subs, len(self.views), vs, self.intr.data_ptr(),
                        self.viewmat.data_ptr())
            self._batch = (key, b, subs, vs)
        return self._batch[1]

    def view_image(self, plane, v):
        """Slice a [C, P] (or [P]) output plane to view v as [C, H, W]."""
        w, h, _ = self.views[v]
        o = self.pixel_offsets[v]
        x = plane[..., o:o + w * h]
        return x.reshape(*x.shape[:-1], h, w)

    def zero_grads(self):
        grads = [{k: torch.zeros_like(sm[k]) for k in PLANES} for sm in self.submaps]
        return grads, torch.zeros_like(self.viewmat)


@dataclass
class Workspace:
    buf: torch.Tensor
    nbytes: int
    max_pairs: int
    params: FmRasterParams
    n_pairs: int = -1
    extra: dict = field(default_factory=dict)


def _outputs(out):
    return FmOutputs(out["rgb"].data_ptr(), out["depth"].data_ptr(), out["normal"].data_ptr(),
                     out["alpha"].data_ptr())


def _grad_structs(grads):
    arr = (FmSurfelGrads * len(grads))()
    for i, g in enumerate(grads):
        for k in PLANES:
            t = g.get(k) if g is not None else None
            if t is not None:
                assert t.is_contiguous() and t.dtype == torch.float32
            setattr(arr[i], k, t.data_ptr() if t is not None else None)
    return arr


class Rasterizer:
    """One fm_ctx on one device."""

    def __init__(self, device=None):
        self.lib = native.load()
        dev = torch.cuda.current_device() if device is None else int(device)
        self.device = dev
        ctx = ctypes.c_void_p()
        st = self.lib.fm_create(ctypes.byref(ctx), dev)
        if st != 0:
            raise native.FmError(st, "fm_create failed")
        self.ctx = ctx

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.lib.fm_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # -- helpers ---------------------------------------------------------
    def check(self, st):
        if st != 0:
            raise native.FmError(st, self.lib.fm_last_error(self.ctx).decode())

    def params(self, alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, rho_max=3.0, near=0.2,
               bg=(0.0, 0.0, 0.0), tile=(16, 16), deterministic=False, overwrite=False, tile_order=0,
               tile_waves=0, lds_depth=0):
        p = FmRasterParams()
        self.lib.fm_default_params(ctypes.byref(p))
        p.alpha_min, p.alpha_max, p.t_min, p.rho_max, p.near_plane = alpha_min, alpha_max, t_min, rho_max, near
        for k in range(3):
            p.bg[k] = bg[k]
        p.tile_w, p.tile_h = tile
        p.deterministic = 1 if deterministic else 0
        p.overwrite = 1 if overwrite else 0
        p.tile_order = int(tile_order)
        p.tile_waves = int(tile_waves)
        p.lds_depth = int(lds_depth)
        return p

    def workspace_size(self, gs, params, max_pairs):
        n = ctypes.c_size_t(0)
        self.check(self.lib.fm_workspace_size(self.ctx, ctypes.byref(gs.batch()), ctypes.byref(params),
                                              int(max_pairs), ctypes.byref(n)))
        return int(n.value)

    def workspace(self, gs, params=None, max_pairs=None):
        params = params or self.params()
        if max_pairs is None:
            ent = sum(int(gs.submaps[s]["opacity"].shape[-1]) for (_, _, s) in gs.views
                      if 0 <= s < len(gs.submaps))
            max_pairs = max(1 << 16, 4 * ent)
        nbytes = self.workspace_size(gs, params, max_pairs)
        buf = torch.empty(nbytes, dtype=torch.uint8, device=gs.intr.device)
        return Workspace(buf, nbytes, int(max_pairs), params)

    def new_outputs(self, gs):
        d = gs.intr.device
        return dict(rgb=torch.empty(3, gs.npx, device=d), depth=torch.empty(gs.npx, device=d),
                    normal=torch.empty(3, gs.npx, device=d), alpha=torch.empty(gs.npx, device=d))

    def query(self, gs, ws):
        """(status, n_pairs, required) of the last forward on ws (synchronous)."""
        n = ctypes.c_int64(0)
        r = ctypes.c_int64(0)
        st = self.lib.fm_query_status(self.ctx, ctypes.byref(gs.batch()), ctypes.byref(ws.params), _ptr(ws.buf),
                                      ws.max_pairs, ctypes.byref(n), ctypes.byref(r))
        if st not in (0, native.FM_ERR_CAPACITY):
            self.check(st)
        return st, int(n.value), int(r.value)

    # -- forward / backward -------------------------------------------------
    def forward_into(self, gs, ws, out, stream=None):
        self.check(self.lib.fm_forward(self.ctx, ctypes.byref(gs.batch()), ctypes.byref(ws.params),
                                       _outputs(out), _ptr(ws.buf), ws.nbytes, ws.max_pairs, _stream(stream)))

    def forward(self, gs, params=None, ws=None, out=None, grow=True):
        """Render every view; grows the pair capacity (synchronising) when it
        overflows.  Returns (outputs, workspace)."""
        params = params or self.params()
        ws = ws or self.workspace(gs, params)
        out = out or self.new_outputs(gs)
        while True:
            self.forward_into(gs, ws, out)
            if not grow:
                return out, ws
            st, n, req = self.query(gs, ws)
            ws.n_pairs = n
            if st == 0:
                return out, ws
            ws = self.workspace(gs, params, max_pairs=int(req * 1.25) + 1024)

    def backward(self, gs, ws, out, g, grads, dviewmat=None, stream=None):
        """Accumulate gradients of the last forward on ws.  g: dict of
        dL/d(rgb, depth, normal, alpha) planes (missing = zero); grads: list
        (per submap) of dicts of gradient tensors (+=)."""
        keep = {k: (g[k].contiguous() if g.get(k) is not None else None)
                for k in ("rgb", "depth", "normal", "alpha")}
        gstruct = FmGradOutputs(*[(keep[k].data_ptr() if keep[k] is not None else None)
                                  for k in ("rgb", "depth", "normal", "alpha")])
        gg = _grad_structs(grads)
        self.check(self.lib.fm_backward(self.ctx, ctypes.byref(gs.batch()), ctypes.byref(ws.params),
                                        _outputs(out), gstruct, _ptr(ws.buf), ws.nbytes, ws.max_pairs, gg,
                                        _ptr(dviewmat), _stream(stream)))
        del keep

    def fwd_bwd_l1(self, gs, ws, out, grads, dviewmat, loss, mask=None, stream=None):
        """Fused forward + L1 loss + backward (adds the loss into `loss`)."""
        ls = FmL1Loss(gs.target_rgb.data_ptr(),
                      gs.target_depth.data_ptr() if gs.target_depth is not None else None,
                      mask.data_ptr() if mask is not None else None, gs.w_rgb,
                      gs.w_depth if gs.target_depth is not None else 0.0)
        gg = _grad_structs(grads)
        self.check(self.lib.fm_fwd_bwd_l1(self.ctx, ctypes.byref(gs.batch()), ctypes.byref(ws.params),
                                          ctypes.byref(ls), _outputs(out), _ptr(loss), gg, _ptr(dviewmat),
                                          _ptr(ws.buf), ws.nbytes, ws.max_pairs, _stream(stream)))

    def fwd_bwd_l1_noalloc(self, gs, params, max_pairs, out, grads, dviewmat, loss, pair_status=None, mask=None,
                           stream=None):
        """fwd_bwd_l1 on the library's static scratch array instead of a
        workspace (fm_fwd_bwd_l1_noalloc).  pair_status: optional int64
        device tensor of 2 (pairs needed, overflow flag)."""
        ls = FmL1Loss(gs.target_rgb.data_ptr(),
                      gs.target_depth.data_ptr() if gs.target_depth is not None else None,
                      mask.data_ptr() if mask is not None else None, gs.w_rgb,
                      gs.w_depth if gs.target_depth is not None else 0.0)
        gg = _grad_structs(grads)
        self.check(self.lib.fm_fwd_bwd_l1_noalloc(self.ctx, ctypes.byref(gs.batch()), ctypes.byref(params),
                                                  ctypes.byref(ls), _outputs(out), _ptr(loss), gg, _ptr(dviewmat),
                                                  int(max_pairs), _ptr(pair_status), _stream(stream)))

    def autotune(self, gs, ws, out, grads, dviewmat, loss, cache_path=None):
        ls = FmL1Loss(gs.target_rgb.data_ptr(),
                      gs.target_depth.data_ptr() if gs.target_depth is not None else None, None, gs.w_rgb,
                      gs.w_depth if gs.target_depth is not None else 0.0)
        chosen = FmRasterParams()
        gg = _grad_structs(grads)
        self.check(self.lib.fm_autotune(self.ctx, ctypes.byref(gs.batch()), ctypes.byref(ws.params),
                                        ctypes.byref(ls), _outputs(out), _ptr(loss), gg, _ptr(dviewmat),
                                        _ptr(ws.buf), ws.nbytes, ws.max_pairs,
                                        cache_path.encode() if cache_path else None, ctypes.byref(chosen),
                                        _stream(None)))
        return chosen

    def pixel_state(self, gs, ws):
        """Per-pixel final transmittance and number of composited surfels of
        the last forward (numpy, synchronous)."""
        import numpy as np
        tf = np.zeros(gs.npx, np.float32)
        nc = np.zeros(gs.npx, np.uint32)
        self.check(self.lib.fm_debug_pixel_state(self.ctx, ctypes.byref(gs.batch()), ctypes.byref(ws.params),
                                                 _ptr(ws.buf), ws.max_pairs, tf.ctypes.data, nc.ctypes.data,
                                                 gs.npx))
        return tf, nc

    def counts(self, gs, ws):
        """(visible entries, kept pairs) of the last forward on ws (synchronous)."""
        nv, nk = ctypes.c_int64(0), ctypes.c_int64(0)
        self.check(self.lib.fm_debug_counts(self.ctx, ctypes.byref(gs.batch()), ctypes.byref(ws.params),
                                            _ptr(ws.buf), ws.max_pairs, ctypes.byref(nv), ctypes.byref(nk)))
        return int(nv.value), int(nk.value)

    def set_timing(self, on=True):
        self.check(self.lib.fm_set_timing(self.ctx, 1 if on else 0))

    PHASES = ("projection", "binning", "zero_grad", "blend", "loss_reduce", "backward_projection")

    def phase_times(self):
        """Milliseconds per phase of the last timed call."""
        ms = (ctypes.c_float * 6)()
        self.check(self.lib.fm_phase_times(self.ctx, ms, 6))
        return dict(zip(self.PHASES, [float(x) for x in ms]))

    def debug_pairs(self, gs, ws):
        """Sorted pair list of the last forward: (tile, surfel, view, tile_start, tile_end) as numpy."""
        import numpy as np
        n = ctypes.c_int64(0)
        tcount = ctypes.c_int64(0)
        self.check(self.lib.fm_tile_count(ctypes.byref(gs.batch()), ctypes.byref(ws.params), ctypes.byref(tcount)))
        self.check(self.lib.fm_debug_pairs(self.ctx, ctypes.byref(gs.batch()), ctypes.byref(ws.params),
                                           _ptr(ws.buf), ws.max_pairs, None, None, None, 0, ctypes.byref(n),
                                           None, None, 0))
        m = int(n.value)
        tile = np.zeros(max(m, 1), np.uint32)
        surf = np.zeros(max(m, 1), np.uint32)
        view = np.zeros(max(m, 1), np.uint32)
        ts = np.zeros(int(tcount.value), np.uint32)
        te = np.zeros(int(tcount.value), np.uint32)
        self.check(self.lib.fm_debug_pairs(self.ctx, ctypes.byref(gs.batch()), ctypes.byref(ws.params),
                                           _ptr(ws.buf), ws.max_pairs, tile.ctypes.data, surf.ctypes.data,
                                           view.ctypes.data, m, ctypes.byref(n), ts.ctypes.data, te.ctypes.data,
                                           int(tcount.value)))
        return tile[:m], surf[:m], view[:m], ts, te


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------

# parameterisation each surfel tensor is stepped in (the rasterizer takes
# activated opacity and linear scales)
ADAM_KINDS = {"mean": native.FM_PARAM_LINEAR, "quat": native.FM_PARAM_LINEAR, "scale": native.FM_PARAM_LOG,
              "opacity": native.FM_PARAM_LOGIT, "color": native.FM_PARAM_LINEAR}
ADAM_LR = {"mean": 1e-3, "quat": 1e-3, "scale": 5e-3, "opacity": 5e-2, "color": 2.5e-3}


class Adam:
    """Fused Adam over the surfel tensors of a GpuScene (fm_adam_step): one
    moment pair per tensor and a device step counter, so a captured graph
    replays consecutive steps.  grads: the per-submap gradient dicts the
    rasterizer accumulates into (their buffers must stay the same); with
    zero_grad the step clears them for the next accumulation."""

    def __init__(self, rast, gs, grads, lr=None, betas=(0.9, 0.999), eps=1e-8, zero_grad=False):
        self.rast = rast
        self.lr = dict(ADAM_LR, **(lr or {}))
        self.m = [{k: torch.zeros_like(sm[k]) for k in PLANES} for sm in gs.submaps]
        self.v = [{k: torch.zeros_like(sm[k]) for k in PLANES} for sm in gs.submaps]
        self.step_count = torch.zeros(1, dtype=torch.int32, device=gs.intr.device)
        self.config = native.FmAdamConfig(betas[0], betas[1], eps, 1 if zero_grad else 0)
        n = len(gs.submaps) * len(PLANES)
        self.tensors = (native.FmAdamTensor * n)()
        i = 0
        for sm, g, m, v in zip(gs.submaps, grads, self.m, self.v):
            for k in PLANES:
                for t in (sm[k], g[k]):
                    assert t.is_contiguous() and t.dtype == torch.float32
                self.tensors[i] = native.FmAdamTensor(sm[k].data_ptr(), g[k].data_ptr(), m[k].data_ptr(),
                                                      v[k].data_ptr(), sm[k].numel(), self.lr[k], ADAM_KINDS[k])
                i += 1
        self.n = n

    def step(self, stream=None):
        self.rast.check(self.rast.lib.fm_adam_step(self.rast.ctx, self.tensors, self.n, ctypes.byref(self.config),
                                                   _ptr(self.step_count), _stream(stream)))


def prune_scores(rast, gs, params=None, tau_rgb=0.1, tau_depth=None, mask=None, ws=None, out=None,
                 stream=None):
    """Error-attributed pruning scores of map fusion (Sec. 3.3) through
    fm_prune_scores: renders the batch, flags the high-error pixels (mean
    absolute RGB error above tau_rgb, or with tau_depth and depth targets
    |D - D*| above tau_depth; or the pixels of the uint8 `mask`) and sums
    every surfel's compositing weight alpha T over them.  Grows the pair
    capacity (synchronising) when it overflows.  Returns (scores: one tensor
    [n] per submap, flags: uint8 [P], outputs, workspace)."""
    params = params or rast.params()
    ws = ws or rast.workspace(gs, params)
    out = out or rast.new_outputs(gs)
    dev = gs.intr.device
    scores = [torch.zeros(int(sm["opacity"].shape[-1]), device=dev) for sm in gs.submaps]
    flags = torch.empty(gs.npx, dtype=torch.uint8, device=dev)
    use_depth = tau_depth is not None and gs.target_depth is not None and mask is None
    spec = native.FmPruneSpec(gs.target_rgb.data_ptr() if gs.target_rgb is not None else None,
                              gs.target_depth.data_ptr() if use_depth else None,
                              mask.data_ptr() if mask is not None else None, flags.data_ptr(),
                              float(tau_rgb), float(tau_depth) if use_depth else 0.0)
    arr = (ctypes.c_void_p * len(scores))(*[t.data_ptr() for t in scores])
    while True:
        rast.check(rast.lib.fm_prune_scores(rast.ctx, ctypes.byref(gs.batch()), ctypes.byref(params),
                                            ctypes.byref(spec), _outputs(out), arr, _ptr(ws.buf), ws.nbytes,
                                            ws.max_pairs, _stream(stream)))
        st, n, req = rast.query(gs, ws)
        ws.n_pairs = n
        if st == 0:
            return scores, flags, out, ws
        ws = rast.workspace(gs, params, max_pairs=int(req * 1.25) + 1024)


def prune_compact(rast, sm, score, tau_prune=0.0, stream=None):
    """The surfels of one submap (dict of planes [C, n]) whose score is not
    above tau_prune, in their original order (fm_prune_compact).  Reads the
    count back (synchronising) and returns dict of planes [C, count]."""
    n = int(sm["opacity"].shape[-1])
    dev = sm["opacity"].device
    outp = {k: torch.empty(CHANNELS[k], max(n, 1), device=dev) for k in PLANES}
    count = torch.zeros(1, dtype=torch.int32, device=dev)
    wsb = torch.empty(max(int(rast.lib.fm_prune_compact_workspace_size(n)), 4), dtype=torch.uint8, device=dev)
    src = FmSurfels(n, *(sm[k].data_ptr() for k in PLANES))
    buf = native.FmSurfelBuffer(*(outp[k].data_ptr() for k in PLANES), n)
    rast.check(rast.lib.fm_prune_compact(rast.ctx, ctypes.byref(src), _ptr(score), float(tau_prune), buf,
                                         _ptr(count), _ptr(wsb), wsb.numel(), _stream(stream)))
    c = int(count.item())
    return {k: (outp[k][:, :c] if CHANNELS[k] > 1 else outp[k][0, :c]).contiguous() for k in PLANES}


class Fusion:
    """Map fusion of per-pixel maps (fm_voxelize_fuse) with an owned
    workspace and output planes sized for the largest frame."""

    def __init__(self, rast, width, height, device="cuda"):
        self.rast = rast
        self.cap = width * height
        n = rast.lib.fm_fusion_workspace_size(width, height)
        self.ws = torch.empty(max(int(n), 4), dtype=torch.uint8, device=device)
        self.out = {k: torch.empty(CHANNELS[k], self.cap, device=device) for k in PLANES}
        self.count = torch.zeros(1, dtype=torch.int32, device=device)

    def run(self, planes, width, height, s, q, t, tau_depth, accum=None, tau_accum=1.0, stream=None):
        """Fuse one map (dict of device planes [C, W*H]); returns the count
        tensor (device) -- the first count entries of self.out are valid."""
        pm = native.FmPixelMap(width, height, *(planes[k].data_ptr() for k in PLANES))
        pose = native.FmSim3(float(s), (ctypes.c_float * 4)(*[float(x) for x in q]),
                             (ctypes.c_float * 3)(*[float(x) for x in t]))
        fp = native.FmFusionParams(float(tau_depth), float(tau_accum))
        buf = native.FmSurfelBuffer(*(self.out[k].data_ptr() for k in PLANES), self.cap)
        self.rast.check(self.rast.lib.fm_voxelize_fuse(self.rast.ctx, ctypes.byref(pm), ctypes.byref(pose),
                                                       ctypes.byref(fp), _ptr(accum), buf, _ptr(self.count),
                                                       _ptr(self.ws), self.ws.numel(), _stream(stream)))
        return self.count


class FusionBatch:
    """Map fusion of several per-pixel maps in one call
    (fm_voxelize_fuse_batch): owned workspace sized for the frames' shapes
    and output planes holding every pixel of every frame."""

    def __init__(self, rast, shapes, device="cuda"):
        self.rast = rast
        self.shapes = [(int(w), int(h)) for (w, h) in shapes]
        self.n = len(self.shapes)
        self.cap = sum(w * h for (w, h) in self.shapes)
        maps = (native.FmPixelMap * self.n)(*[native.FmPixelMap(w, h, None, None, None, None, None)
                                              for (w, h) in self.shapes])
        nbytes = rast.lib.fm_fusion_batch_workspace_size(maps, self.n)
        self.ws = torch.empty(max(int(nbytes), 4), dtype=torch.uint8, device=device)
        self.out = {k: torch.empty(CHANNELS[k], self.cap, device=device) for k in PLANES}
        self.offsets = torch.zeros(self.n + 1, dtype=torch.int32, device=device)

    def run(self, frames, tau_depth, accums=None, tau_accum=1.0, stream=None):
        """frames: list of (planes, s, q, t) with planes a dict of device
        [C, W*H] tensors, in the order of the shapes; accums: list of device
        gate maps (or None entries) or None.  Returns the offsets tensor
        (device, n + 1): frame f's survivors are out[:, offsets[f]:offsets[f+1]]."""
        assert len(frames) == self.n
        maps = (native.FmPixelMap * self.n)()
        poses = (native.FmSim3 * self.n)()
        for i, ((planes, s, q, t), (w, h)) in enumerate(zip(frames, self.shapes)):
            maps[i] = native.FmPixelMap(w, h, *(planes[k].data_ptr() for k in PLANES))
            poses[i] = native.FmSim3(float(s), (ctypes.c_float * 4)(*[float(x) for x in q]),
                                     (ctypes.c_float * 3)(*[float(x) for x in t]))
        acc = None
        if accums is not None:
            acc = (ctypes.c_void_p * self.n)(*[(a.data_ptr() if a is not None else None) for a in accums])
        fp = native.FmFusionParams(float(tau_depth), float(tau_accum))
        buf = native.FmSurfelBuffer(*(self.out[k].data_ptr() for k in PLANES), self.cap)
        self.rast.check(self.rast.lib.fm_voxelize_fuse_batch(
            self.rast.ctx, maps, poses, self.n, ctypes.byref(fp), acc, buf, _ptr(self.offsets), _ptr(self.ws),
            self.ws.numel(), _stream(stream)))
        return self.offsets


def sim3_table(deltas, device="cuda"):
    """Device table of fm_sim3 records from host (s, q(w,x,y,z), t) triples,
    one per keyframe, for warp_keyframes."""
    arr = (native.FmSim3 * max(1, len(deltas)))()
    for k, (s, q, t) in enumerate(deltas):
        arr[k] = native.FmSim3(float(s), (ctypes.c_float * 4)(*[float(x) for x in q]),
                               (ctypes.c_float * 3)(*[float(x) for x in t]))
    return torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).to(device), len(deltas)


def warp_keyframes(rast, surfels, keyframe, table, stream=None):
    """Loop-correction warp in place (fm_warp_keyframes): surfels holds the
    device planes mean [3, n], quat [4, n], scale [2, n]; keyframe is a
    device int32 [n] binding; table = sim3_table(...) (device records and
    their count).  Primitives bound outside the table are left alone."""
    rec, n_kf = table
    n = int(keyframe.numel())
    rast.check(rast.lib.fm_warp_keyframes(rast.ctx, _ptr(surfels["mean"]), _ptr(surfels["quat"]),
                                          _ptr(surfels["scale"]), _ptr(keyframe), n, _ptr(rec), n_kf,
                                          _stream(stream)))


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rast, gs, params, *flat):
        out, ws = rast.forward(gs, params)
        ctx.rast, ctx.gs, ctx.ws, ctx.out = rast, gs, ws, out
        return out["rgb"], out["depth"], out["normal"], out["alpha"]

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_normal, g_alpha):
        gs = ctx.gs
        grads, dvm = gs.zero_grads()
        g = dict(rgb=g_rgb, depth=g_depth, normal=g_normal, alpha=g_alpha)
        ctx.rast.backward(gs, ctx.ws, ctx.out, g, grads, dvm)
        flat = []
        for gr in grads:
            flat += [gr[k] for k in PLANES]
        return (None, None, None, *flat, dvm)


def render(rast, submaps, views, intr, viewmat, params=None):
    """Differentiable render of a batch.  submaps: list of dicts of
    float32 CUDA tensors (mean[3,n], quat[4,n], scale[2,n], opacity[n],
    color[3,n]); views: list of (W, H, submap); intr [V,4]; viewmat [V,12].
    Returns planes (rgb[3,P], depth[P], normal[3,P], alpha[P]) whose backward
    yields gradients for every surfel plane and for viewmat."""
    gs = GpuScene([{k: sm[k].detach() for k in PLANES} for sm in submaps], views, intr.detach(),
                  viewmat.detach())
    flat = []
    for sm in submaps:
        flat += [sm[k] for k in PLANES]
    return _RenderFn.apply(rast, gs, params or rast.params(), *flat, viewmat)
