"""FP64 CPU oracle for the 2DGS surfel rasterizer (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  It shares no code with the HIP path: the C source
``fm_oracle.c`` is compiled on its own with gcc, and the loss below is
written out from its definition.

Parameters are rounded to float32 before use, so the oracle's FP64 decisions
compare against exactly the thresholds the float32 API carries.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fm_oracle.c")
_LIB = os.path.join(_HERE, "libfm_oracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (OpenMP, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lm"]
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("t_min", ctypes.c_double), ("rho_max", ctypes.c_double),
                ("near_z", ctypes.c_double), ("bg", ctypes.c_double * 3),
                ("margin", ctypes.c_double), ("margin_t", ctypes.c_double),
                ("cond_eps", ctypes.c_double), ("cond_tol", ctypes.c_double),
                ("prefilter", ctypes.c_int), ("n_threads", ctypes.c_int)]


DEFAULTS = dict(alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, rho_max=3.0, near=0.2,
                bg=(0.0, 0.0, 0.0), margin=1e-5, margin_t=2e-4, cond_eps=2e-7, cond_tol=2e-5,
                prefilter=1, n_threads=0)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _params(**kw):
    d = dict(DEFAULTS)
    d.update(kw)
    f32 = lambda v: float(np.float32(v))
    p = _Params()
    p.alpha_min = f32(d["alpha_min"])
    p.alpha_max = f32(d["alpha_max"])
    p.t_min = f32(d["t_min"])
    p.rho_max = f32(d["rho_max"])
    p.near_z = f32(d["near"])
    for k in range(3):
        p.bg[k] = f32(d["bg"][k])
    p.margin = float(d["margin"])
    p.margin_t = float(d["margin_t"])
    p.cond_eps = float(d["cond_eps"])
    p.cond_tol = float(d["cond_tol"])
    p.prefilter = int(d["prefilter"])
    p.n_threads = int(d["n_threads"])
    return p


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a, t=ctypes.c_float):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _surf_args(sm):
    arrs = [_f32(sm[k]) for k in ("mean", "quat", "scale", "opacity", "color")]
    n = arrs[3].shape[-1]
    return n, arrs


def render_view(sm, w, h, intr, viewmat, **kw):
    """Forward of one view.  Returns a dict of float64 planes (rgb[3,WH],
    depth[WH], normal[3,WH], alpha[WH], t_final[WH]), n_contrib[WH],
    flags[WH] and n_useful."""
    L = lib()
    n, arrs = _surf_args(sm)
    intr = _f32(intr)
    vm = _f32(viewmat)
    npx = w * h
    rgb = np.zeros((3, npx)); depth = np.zeros(npx); normal = np.zeros((3, npx))
    alpha = np.zeros(npx); tf = np.zeros(npx)
    nc = np.zeros(npx, np.int32); fl = np.zeros(npx, np.uint8)
    nu = ctypes.c_int64(0)
    p = _params(**kw)
    D = ctypes.c_double
    rc = L.orc_render(ctypes.c_int(n), *[_ptr(a) for a in arrs], ctypes.c_int(w), ctypes.c_int(h),
                      _ptr(intr), _ptr(vm), ctypes.byref(p), _ptr(rgb, D), _ptr(depth, D),
                      _ptr(normal, D), _ptr(alpha, D), _ptr(tf, D), _ptr(nc, ctypes.c_int32),
                      _ptr(fl, ctypes.c_uint8), ctypes.byref(nu))
    if rc != 0:
        raise RuntimeError("oracle render failed")
    return dict(rgb=rgb, depth=depth, normal=normal, alpha=alpha, t_final=tf, n_contrib=nc,
                flags=fl.astype(bool), n_useful=int(nu.value))


def backward_view(sm, w, h, intr, viewmat, g, grads=None, **kw):
    """Backward of one view.  g holds dL/d(outputs) planes (rgb, depth,
    normal, alpha).  Gradients are added into ``grads`` (created if None):
    mean[3,n], quat[4,n], scale[2,n], opacity[n], color[3,n], viewmat[12]."""
    L = lib()
    n, arrs = _surf_args(sm)
    if grads is None:
        grads = dict(mean=np.zeros((3, n)), quat=np.zeros((4, n)), scale=np.zeros((2, n)),
                     opacity=np.zeros(n), color=np.zeros((3, n)), viewmat=np.zeros(12))
    npx = w * h
    D = ctypes.c_double
    gg = [np.ascontiguousarray(np.asarray(g[k], np.float64).reshape(-1)) for k in
          ("rgb", "depth", "normal", "alpha")]
    assert gg[0].size == 3 * npx and gg[1].size == npx and gg[2].size == 3 * npx and gg[3].size == npx
    p = _params(**kw)
    rc = L.orc_render_backward(ctypes.c_int(n), *[_ptr(a) for a in arrs], ctypes.c_int(w),
                               ctypes.c_int(h), _ptr(_f32(intr)), _ptr(_f32(viewmat)), ctypes.byref(p),
                               *[_ptr(a, D) for a in gg],
                               *[_ptr(grads[k], D) for k in ("mean", "quat", "scale", "opacity",
                                                             "color", "viewmat")])
    if rc != 0:
        raise RuntimeError("oracle backward failed")
    return grads


def bin_view(sm, w, h, intr, viewmat, tile_w=16, tile_h=16, cap=None, **kw):
    """Tile binning of one view: per-surfel tile rects and depth-key bits,
    the pair list sorted by (tile, depth key, index) with tile ranges, and
    per pair whether the surfel reaches a pixel of the tile (passes the
    support and opacity tests at one of its pixel centres)."""
    L = lib()
    n, arrs = _surf_args(sm)
    rect = np.zeros((n, 4), np.int32)
    kappa = np.zeros(n, np.uint32)
    npairs = ctypes.c_int64(0)
    tx, ty = (w + tile_w - 1) // tile_w, (h + tile_h - 1) // tile_h
    ts = np.zeros(tx * ty, np.uint32); te = np.zeros(tx * ty, np.uint32)
    p = _params(**kw)
    args_head = [ctypes.c_int(n), *[_ptr(a) for a in arrs], ctypes.c_int(w), ctypes.c_int(h),
                 _ptr(_f32(intr)), _ptr(_f32(viewmat)), ctypes.byref(p), ctypes.c_int(tile_w),
                 ctypes.c_int(tile_h), _ptr(rect, ctypes.c_int32), _ptr(kappa, ctypes.c_uint32),
                 ctypes.byref(npairs)]
    c = 1 if cap is None else cap

    def run(c):
        pt = np.zeros(max(c, 1), np.uint32); ps = np.zeros(max(c, 1), np.uint32)
        pr = np.zeros(max(c, 1), np.uint8)
        rc = L.orc_bin(*args_head, _ptr(pt, ctypes.c_uint32), _ptr(ps, ctypes.c_uint32),
                       ctypes.c_int64(c), _ptr(ts, ctypes.c_uint32), _ptr(te, ctypes.c_uint32),
                       _ptr(pr, ctypes.c_uint8))
        return rc, pt, ps, pr

    rc, pt, ps, pr = run(c)
    if rc == 2 and cap is None:
        rc, pt, ps, pr = run(int(npairs.value))
    if rc != 0:
        raise RuntimeError(f"oracle binning failed ({rc})")
    m = int(npairs.value)
    return dict(rect=rect, kappa=kappa, n_pairs=m, pair_tile=pt[:m].copy(), pair_surf=ps[:m].copy(),
                pair_reached=pr[:m].astype(bool), tile_start=ts, tile_end=te, tiles=(tx, ty))


def project(sm, w, h, intr, viewmat, **kw):
    """Per-surfel culling summary: valid flag, FP64 depth, pixel bbox."""
    L = lib()
    n, arrs = _surf_args(sm)
    valid = np.zeros(n, np.int32); depth = np.zeros(n); bb = np.zeros((n, 4), np.int32)
    p = _params(**kw)
    L.orc_project(ctypes.c_int(n), *[_ptr(a) for a in arrs], ctypes.c_int(w), ctypes.c_int(h),
                  _ptr(_f32(intr)), _ptr(_f32(viewmat)), ctypes.byref(p),
                  _ptr(valid, ctypes.c_int32), _ptr(depth, ctypes.c_double), _ptr(bb, ctypes.c_int32))
    return dict(valid=valid.astype(bool), depth=depth, pix_bbox=bb)


# ---------------------------------------------------------------------------
# whole scenes (several views / submaps)
# ---------------------------------------------------------------------------

def render_scene(scene, views=None, **kw):
    """Forward of every view (or the listed ones); planes concatenated view
    after view in the scene's pixel order (only the listed views)."""
    views = range(scene.n_views) if views is None else views
    outs = []
    for v in views:
        w, h, s = scene.views[v]
        outs.append(render_view(scene.submaps[s], w, h, scene.intr[v], scene.viewmat[v], **kw))
    cat = {}
    for k in ("rgb", "normal"):
        cat[k] = np.concatenate([o[k] for o in outs], axis=1)
    for k in ("depth", "alpha", "t_final", "n_contrib", "flags"):
        cat[k] = np.concatenate([o[k] for o in outs])
    cat["n_useful"] = sum(o["n_useful"] for o in outs)
    return cat


def l1_loss(scene, out, views=None, mask=None):
    """Render loss of one batch: for each view, w_rgb * mean |I - I*| over
    pixels and channels plus w_depth * mean |D - D*| over pixels, summed over
    views (the L1 form of the paper's render term, Sec. 3.1).  Returns the
    loss and dL/d(outputs) planes.  ``mask`` (per pixel, optional) zeroes
    pixels in both the loss and its gradient; the means still divide by the
    full pixel count."""
    views = list(range(scene.n_views)) if views is None else list(views)
    offs = scene.pixel_offsets
    sel = np.concatenate([np.arange(offs[v], offs[v] + scene.view_pixels(v)) for v in views])
    t_rgb = scene.target_rgb[:, sel].astype(np.float64)
    t_d = scene.target_depth[sel].astype(np.float64) if scene.target_depth is not None else None
    npx_each = np.concatenate([np.full(scene.view_pixels(v), scene.view_pixels(v)) for v in views])
    m = np.ones(sel.size) if mask is None else np.asarray(mask, np.float64)
    diff = out["rgb"] - t_rgb
    loss = scene.w_rgb * np.sum(m * np.abs(diff) / (3.0 * npx_each))
    g_rgb = scene.w_rgb * m * np.sign(diff) / (3.0 * npx_each)
    g_d = np.zeros(sel.size)
    if t_d is not None and scene.w_depth != 0.0:
        dd = out["depth"] - t_d
        loss += scene.w_depth * np.sum(m * np.abs(dd) / npx_each)
        g_d = scene.w_depth * m * np.sign(dd) / npx_each
    return float(loss), dict(rgb=g_rgb, depth=g_d, normal=np.zeros((3, sel.size)),
                             alpha=np.zeros(sel.size))


def backward_scene(scene, g, views=None, **kw):
    """Backward of the listed views; g planes in the same concatenated
    order as render_scene.  Returns per-submap gradient dicts and the
    per-view viewmat gradients [V,12] (zero rows for unlisted views)."""
    views = list(range(scene.n_views)) if views is None else list(views)
    grads = []
    for sm in scene.submaps:
        n = sm["opacity"].shape[0]
        grads.append(dict(mean=np.zeros((3, n)), quat=np.zeros((4, n)), scale=np.zeros((2, n)),
                          opacity=np.zeros(n), color=np.zeros((3, n)), viewmat=np.zeros(12)))
    dvm = np.zeros((scene.n_views, 12))
    off = 0
    for v in views:
        w, h, s = scene.views[v]
        npx = w * h
        gv = {k: (g[k][:, off:off + npx] if g[k].ndim == 2 else g[k][off:off + npx])
              for k in ("rgb", "depth", "normal", "alpha")}
        grads[s]["viewmat"][:] = 0.0
        backward_view(scene.submaps[s], w, h, scene.intr[v], scene.viewmat[v], gv, grads[s], **kw)
        dvm[v] = grads[s]["viewmat"]
        off += npx
    for gr in grads:
        gr.pop("viewmat")
    return grads, dvm
