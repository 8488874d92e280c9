"""GPU parity where depth keys tie (the tie-break reading: candidates are
ordered by (fp32 depth key, surfel index)).

Random float depths practically never tie, so two scenes make ties on
purpose: a stack of fronto-parallel surfels with bit-equal depths listed out
of index order (closed form of Eq. 1 at the pixel they share), and a random
scene whose centre depths are quantised to multiples of 1/4 and seen from
cameras without rotation, so the camera-space depth equals the quantised
value exactly and hundreds of surfels share each key.  Pair lists are
compared with the oracle's on every pair, images and gradients at the usual
tolerances."""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_03092_amd import scenes
from paper_2604_03092_amd.raster import GpuScene, Rasterizer
from tests.gpu_util import (assert_grad_close, assert_images_close, assert_pairs_match, random_upstream,
                            to_np)

pytestmark = pytest.mark.gpu

TILES = [(16, 16), (8, 8), (16, 8), (32, 8), (32, 32)]


@pytest.fixture(scope="module")
def rast():
    return Rasterizer()


def _say(msg):
    print(msg, flush=True)


def _surfel(mu, sigma, color, scale=0.5):
    f = lambda a: np.asarray(a, np.float32).reshape(-1, 1)
    return dict(mean=f(mu), quat=f([1, 0, 0, 0]), scale=f([scale, scale]),
                opacity=np.asarray([sigma], np.float32), color=f(color))


def _tie_stack_scene():
    """Indices 0, 2 and 4 share the depth 3.0; index 1 lies in front at 2.0,
    index 3 behind at 4.0: compositing order 1, 0, 2, 4, 3 at every pixel."""
    parts = [_surfel([0, 0, 3.0], 0.3, [1, 0, 0]), _surfel([0, 0, 2.0], 0.2, [0, 0, 0]),
             _surfel([0, 0, 3.0], 0.6, [0, 1, 0]), _surfel([0, 0, 4.0], 0.5, [1, 1, 1]),
             _surfel([0, 0, 3.0], 0.45, [0, 0, 1])]
    sm = {k: np.concatenate([p[k] for p in parts], axis=-1) for k in parts[0]}
    intr = np.array([[20, 20, 8.5, 8.5]], np.float32)
    vm = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
    sc = scenes.Scene("tie_stack", [sm], [(16, 16, 0)], intr, vm, w_rgb=1.0, w_depth=0.0)
    return sc, [1, 0, 2, 4, 3]


def test_tie_stack_closed_form(rast):
    sc, order = _tie_stack_scene()
    sm = sc.submaps[0]
    gs = GpuScene.from_scene(sc)
    for tile in TILES:
        out, ws = rast.forward(gs, rast.params(tile=tile))
        torch.cuda.synchronize()
        q = 8 * 16 + 8   # pixel (8, 8): (u, v) = (0, 0) on every surfel
        T, rgb, d = 1.0, np.zeros(3), 0.0
        for i in order:
            a = float(sm["opacity"][i])
            rgb += sm["color"][:, i].astype(np.float64) * a * T
            d += float(sm["mean"][2, i]) * a * T
            T *= 1.0 - a
        got = to_np(out["rgb"])[:, q]
        assert np.abs(got - rgb).max() <= 1e-6, (tile, got, rgb)
        assert abs(float(out["depth"][q]) - d) <= 1e-5
        ref = oracle.render_scene(sc)
        assert_images_close(out, ref, ~ref["flags"], what=f"tie stack {tile}")
        b = oracle.bin_view(sm, 16, 16, sc.intr[0], sc.viewmat[0], tile_w=tile[0], tile_h=tile[1])
        t, s, _, ts, te = rast.debug_pairs(gs, ws)
        assert_pairs_match(b, t, s, ts, te)
        tile_of_px = (8 // tile[1]) * ((16 + tile[0] - 1) // tile[0]) + 8 // tile[0]
        assert list(s[ts[tile_of_px]:te[tile_of_px]]) == order, tile


def _quantised_scene():
    """5,000 surfels of config-0 laws with centre depths rounded to multiples
    of 1/4 (17 keys between 2 and 6), two views related by a translation."""
    sc = scenes.random_scene(57, 5000, 96, 72, n_views=1, scale_lo=0.03, scale_hi=0.2)
    sm = sc.submaps[0]
    sm["mean"][2] = (np.round(sm["mean"][2] * 4.0) / 4.0).astype(np.float32)
    vm = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0],
                   [1, 0, 0, 0.125, 0, 1, 0, -0.0625, 0, 0, 1, 0]], np.float32)
    intr = np.tile(sc.intr[:1], (2, 1))
    out = scenes.Scene("quantised_depth", [sm], [(96, 72, 0)] * 2, intr, vm, w_rgb=1.0, w_depth=0.1)
    rng = np.random.default_rng(58)
    out.target_rgb = rng.random((3, out.total_pixels)).astype(np.float32)
    out.target_depth = rng.uniform(1.0, 8.0, out.total_pixels).astype(np.float32)
    return out


def test_quantised_depths_pairs_images_gradients(rast):
    sc = _quantised_scene()
    sm = sc.submaps[0]
    z = sm["mean"][2]
    _, counts = np.unique(z, return_counts=True)
    assert counts.max() > 200            # many surfels share each key
    gs = GpuScene.from_scene(sc)
    ref = oracle.render_scene(sc)
    keep = ~ref["flags"]
    assert keep.mean() > 0.98
    for tile in TILES:
        _say(f"quantised depths tile={tile}")
        out, ws = rast.forward(gs, rast.params(tile=tile))
        torch.cuda.synchronize()
        assert_images_close(out, ref, keep, what=f"quantised {tile}")
        t, s, view, ts, te = rast.debug_pairs(gs, ws)
        tiles_per_view = len(ts) // sc.n_views
        for v in range(sc.n_views):
            b = oracle.bin_view(sm, 96, 72, sc.intr[v], sc.viewmat[v], tile_w=tile[0], tile_h=tile[1])
            sel = view == v
            lo = v * tiles_per_view
            assert_pairs_match(b, t[sel] - lo, s[sel], ts[lo:lo + tiles_per_view], te[lo:lo + tiles_per_view])
    # gradients through the adjoint (16x16) against the oracle
    out, ws = rast.forward(gs, rast.params(tile=(16, 16)))
    g = random_upstream(np.random.default_rng(59), gs.npx, keep)
    gt = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in g.items()}
    grads, dvm = gs.zero_grads()
    rast.backward(gs, ws, out, gt, grads, dvm)
    torch.cuda.synchronize()
    rg, rdvm = oracle.backward_scene(sc, g)
    for k in ("mean", "quat", "scale", "opacity", "color"):
        assert_grad_close(to_np(grads[0][k]), rg[0][k], f"quantised.{k}")
    assert_grad_close(to_np(dvm), rdvm, "quantised.viewmat")
