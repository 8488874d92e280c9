"""GPU checks at the benchmark sizes (16 x 640x480 over 300k surfels; 1M
shared surfels; uneven multi-submap batches; per-pixel maps), in the launch
configuration bench.py times (fused batch, 16x16 tiles), on outputs the
oracle can compute view by view; gradients at these sizes are checked through
properties (batch = sum of views) and at reduced sizes against the oracle."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2604_03092_amd import scenes
from paper_2604_03092_amd.raster import GpuScene, Rasterizer
from tests.gpu_util import assert_grad_close, assert_images_close, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rast():
    return Rasterizer()


def _say(msg):
    print(msg, flush=True)


def _fused(rast, gs, params=None, mask=None):
    params = params or rast.params()
    out, ws = rast.forward(gs, params)
    ws = rast.workspace(gs, params, max_pairs=ws.n_pairs + 4096)
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    loss = torch.zeros(1, device="cuda")
    rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss, mask=mask)
    torch.cuda.synchronize()
    assert rast.query(gs, ws)[0] == 0
    return out, grads, dvm, float(loss), ws


def _view_scene(sc, v):
    w, h, s = sc.views[v]
    o = sc.pixel_offsets[v]
    return scenes.Scene(f"{sc.name}_v{v}", sc.submaps, [sc.views[v]], sc.intr[v:v + 1], sc.viewmat[v:v + 1],
                        sc.target_rgb[:, o:o + w * h],
                        None if sc.target_depth is None else sc.target_depth[o:o + w * h], sc.w_rgb, sc.w_depth)


def _check_sampled_views(rast, sc, views, params=None):
    gs = GpuScene.from_scene(sc)
    _say(f"{sc.name}: fused batch of {gs.n_views} views")
    out, grads, dvm, loss, ws = _fused(rast, gs, params)
    for v in views:
        _say(f"{sc.name}: oracle view {v}")
        ref = oracle.render_scene(_view_scene(sc, v))
        keep = ~ref["flags"]
        assert keep.mean() > 0.99
        o = gs.pixel_offsets[v]
        sl = slice(o, o + sc.view_pixels(v))
        got = {k: x[..., sl] for k, x in out.items()}
        assert_images_close(got, ref, keep, what=f"{sc.name} view {v}")
    return gs, out, grads, dvm, loss


def test_headline_batch_sampled_views_and_loss(rast):
    sc = scenes.headline()
    gs, out, grads, dvm, loss = _check_sampled_views(rast, sc, [0, 9])
    # loss of the whole batch against the oracle's (view by view)
    _say("headline: oracle loss over all views")
    ref_loss = 0.0
    for v in range(sc.n_views):
        one = _view_scene(sc, v)
        ref_loss += oracle.l1_loss(one, oracle.render_scene(one))[0]
    assert abs(loss - ref_loss) <= 2e-5 * ref_loss, (loss, ref_loss)


def test_headline_batch_gradients_equal_sum_of_views(rast):
    """Property at full size: the fused 16-view gradients equal the sum of the
    16 single-view fused gradients (same kernels, different batching)."""
    sc = scenes.headline()
    gs = GpuScene.from_scene(sc)
    _say("headline gradients: batch")
    _, grads, dvm, loss, _ = _fused(rast, gs)
    acc, _ = gs.zero_grads()
    tot = 0.0
    for v in range(sc.n_views):
        gv = GpuScene.from_scene(_view_scene(sc, v))
        gv.submaps = gs.submaps
        gv._batch = None
        _, g1, d1, l1, _ = _fused(rast, gv)
        for k in acc[0]:
            acc[0][k] += g1[0][k]
        assert torch.allclose(d1[0], dvm[v], rtol=2e-4, atol=1e-6 * float(dvm.abs().max()))
        tot += l1
    assert abs(tot - loss) <= 1e-5 * loss
    for k in acc[0]:
        assert_grad_close(to_np(grads[0][k]), to_np(acc[0][k]), f"headline.{k}", rel=1e-4)


def test_config2_sampled_views(rast):
    _check_sampled_views(rast, scenes.config2(), [3])


def test_config3_sampled_views(rast):
    sc = scenes.config3()
    big = max(range(sc.n_views), key=lambda v: sc.views[v][0])
    _check_sampled_views(rast, sc, [0, big])


def test_config4_sampled_views_8x8(rast):
    sc = scenes.config4()
    _check_sampled_views(rast, sc, [5], params=rast.params(tile=(8, 8)))


def test_config4_reduced_gradients(rast):
    """Per-pixel surfel maps (config-4 laws) at a size the oracle
    differentiates in seconds: 3 frames of 130x98."""
    sc = scenes.config4(n_frames=3, w=130, h=98)
    gs = GpuScene.from_scene(sc)
    ref = oracle.render_scene(sc)
    near = np.any(np.abs(ref["rgb"] - sc.target_rgb) < 5e-4, axis=0) | (np.abs(ref["depth"] - sc.target_depth) < 5e-4)
    keep = ~(ref["flags"] | near)
    mask = torch.from_numpy(keep.astype(np.uint8)).cuda()
    _say("config4 reduced: fused")
    out, grads, dvm, loss, _ = _fused(rast, gs, rast.params(tile=(8, 8)), mask=mask)
    assert_images_close(out, ref, ~ref["flags"], what="config4 reduced")
    L, g = oracle.l1_loss(sc, ref, mask=keep)
    assert abs(loss - L) <= 1e-5 * L
    rg, rdvm = oracle.backward_scene(sc, g)
    for s in range(len(sc.submaps)):
        for k in ("mean", "quat", "scale", "opacity", "color"):
            assert_grad_close(to_np(grads[s][k]), rg[s][k], f"config4[{s}].{k}")
    assert_grad_close(to_np(dvm), rdvm, "config4.viewmat")


def test_autotune_and_cache(rast, tmp_path):
    sc = scenes.random_scene(21, 40000, 320, 240, n_views=2, scale_lo=0.02, scale_hi=0.1)
    gs = GpuScene.from_scene(sc)
    p8 = rast.params(tile=(8, 8))
    out, ws = rast.forward(gs, p8)
    ws = rast.workspace(gs, p8, max_pairs=ws.n_pairs + 4096)
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    loss = torch.zeros(1, device="cuda")
    path = str(tmp_path / "tune.json")
    _say("autotune")
    chosen = rast.autotune(gs, ws, out, grads, dvm, loss, cache_path=path)
    assert (chosen.tile_w, chosen.tile_h) in [(16, 16), (8, 8), (16, 8), (32, 8), (32, 32)]
    assert chosen.tile_order in (1, 2)
    assert chosen.tile_waves in (1, 2) and chosen.lds_depth in (32, 64, 128)
    data = json.load(open(path))
    key, val = list(data.items())[0]
    assert key.startswith("gfx950")   # the cache is keyed by the device's architecture
    assert val == [chosen.tile_w, chosen.tile_h, chosen.tile_order, chosen.tile_waves, chosen.lds_depth]
    # a fresh context reads the cache; tile 0x0 then means "the tuned shape"
    r2 = Rasterizer()
    chosen2 = r2.autotune(gs, ws, out, grads, dvm, loss, cache_path=path)
    assert (chosen2.tile_w, chosen2.tile_h, chosen2.tile_order, chosen2.tile_waves, chosen2.lds_depth) == (
        chosen.tile_w, chosen.tile_h, chosen.tile_order, chosen.tile_waves, chosen.lds_depth)
    auto = r2.params(tile=(0, 0))
    o2, _ = r2.forward(gs, auto)
    ref, _ = r2.forward(gs, r2.params(tile=(chosen.tile_w, chosen.tile_h)))
    for k in ref:
        assert torch.equal(o2[k], ref[k])
