"""Map-fusion pruning in the oracle (test infrastructure only; same rules as
the rest of this package: only tests, the smoke check and the benchmark's
CPU-baseline leg may use it).

The backend first prunes the global map: it renders the map from the new
keyframe's pose and removes every primitive that contributes to pixels with
a high RGB or depth reconstruction error (Sec. 3.3, "Map Fusion").  Written
out from that description:

  * error_mask -- a pixel is high-error when the mean over its three
    channels of |I - I*| exceeds tau_rgb, or, with a depth target, when
    |D - D*| exceeds tau_depth (D is the depth sum of Eq. 1);
  * contribution_scores -- a surfel's score is its total compositing weight
    alpha T (its share in Eq. 1) over the high-error pixels of the view;
  * prune_keep -- a surfel is kept when its score does not exceed tau_prune
    (tau_prune = 0 removes every surfel that contributes at all).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _f32, _params, _ptr, _surf_args, lib


def error_mask(rgb, depth, target_rgb, target_depth=None, tau_rgb=0.1, tau_depth=None):
    """High-error pixels in FP64 from the definition.  rgb / target_rgb:
    [3, P]; depth / target_depth: [P] (depth is used when target_depth and
    tau_depth are given).  Returns a bool array [P]."""
    e = np.mean(np.abs(np.asarray(rgb, np.float64) - np.asarray(target_rgb, np.float64)), axis=0)
    m = e > tau_rgb
    if target_depth is not None and tau_depth is not None:
        m |= np.abs(np.asarray(depth, np.float64) - np.asarray(target_depth, np.float64)) > tau_depth
    return m


def error_mask_f32(rgb, depth, target_rgb, target_depth=None, tau_rgb=0.1, tau_depth=None):
    """The same criterion taken in float32 in a fixed order, for float32
    renderings: d_c = I_c - I*_c, e = (|d_0| + |d_1|) + |d_2|, high when
    e / 3 > tau_rgb (each step rounded to float32), or |D - D*| > tau_depth.
    A decision that floating point takes is compared in the precision the
    GPU takes it in."""
    f = np.float32
    d = np.asarray(rgb, f) - np.asarray(target_rgb, f)
    e = (np.abs(d[0]) + np.abs(d[1])) + np.abs(d[2])
    m = (e / f(3.0)) > f(tau_rgb)
    if target_depth is not None and tau_depth is not None:
        m |= np.abs(np.asarray(depth, f) - np.asarray(target_depth, f)) > f(tau_depth)
    return m


def contribution_scores_view(sm, w, h, intr, viewmat, mask, score=None, **kw):
    """Adds into score[n] (created if None) every surfel's sum of alpha T over
    the pixels of one view where mask is set (FP64)."""
    L = lib()
    n, arrs = _surf_args(sm)
    if score is None:
        score = np.zeros(n)
    m = np.ascontiguousarray(np.asarray(mask).reshape(-1).astype(np.uint8))
    assert m.size == w * h
    p = _params(**kw)
    rc = L.orc_contrib_scores(ctypes.c_int(n), *[_ptr(a) for a in arrs], ctypes.c_int(w), ctypes.c_int(h),
                              _ptr(_f32(intr)), _ptr(_f32(viewmat)), ctypes.byref(p), _ptr(m, ctypes.c_uint8),
                              _ptr(score, ctypes.c_double))
    if rc != 0:
        raise RuntimeError("oracle contribution scores failed")
    return score


def contribution_scores(scene, mask, views=None, **kw):
    """Per-submap scores over the listed views (all by default); mask covers
    the listed views' pixels concatenated in order."""
    views = list(range(scene.n_views)) if views is None else list(views)
    scores = [np.zeros(sm["opacity"].shape[0]) for sm in scene.submaps]
    mask = np.asarray(mask).reshape(-1)
    off = 0
    for v in views:
        w, h, s = scene.views[v]
        contribution_scores_view(scene.submaps[s], w, h, scene.intr[v], scene.viewmat[v],
                                 mask[off:off + w * h], scores[s], **kw)
        off += w * h
    return scores


def prune_keep(score, tau_prune=0.0):
    """Indices of the surfels that stay, in their original order: those whose
    score does not exceed tau_prune (compared in the score's precision)."""
    score = np.asarray(score)
    return np.nonzero(~(score > score.dtype.type(tau_prune)))[0]


def prune_surfels(sm, score, tau_prune=0.0):
    """The surfel planes without the removed surfels (order kept)."""
    keep = prune_keep(score, tau_prune)
    return {k: np.ascontiguousarray(v[..., keep]) for k, v in sm.items()}
