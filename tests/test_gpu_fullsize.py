"""Oracle parity of the fused forward + L1 + backward kernel at full size, in
the launch configuration the benchmark times (16x16 tiles, tiles taken
longest list first, gradients stored), plus the non-default raster
parameters and the batch sizes that take the chunked descriptor path.

Full-size batches run whole on the GPU; the loss mask keeps only the pixels
of the views the oracle renders (and, on those, only pixels whose decisions
and L1 signs are robust: the oracle's margin flags and |I - I*| < 5e-4 are
masked on both sides), so every surfel and pose gradient of the batch is
compared element by element with the oracle's gradient of the same masked
loss.  Each case prints its worst errors on a line starting with PARITY."""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_03092_amd import scenes
from paper_2604_03092_amd.raster import GpuScene, Rasterizer
from tests.gpu_util import (assert_grad_close, assert_images_close, grad_errors, random_upstream, to_np)

pytestmark = pytest.mark.gpu

PLANES = ("mean", "quat", "scale", "opacity", "color")


@pytest.fixture(scope="module")
def rast():
    return Rasterizer()


def _say(msg):
    print(msg, flush=True)


def _bench_params(rast, **kw):
    """The benchmark's launch: 16x16 tiles, longest list first, stored gradients."""
    return rast.params(tile=(16, 16), tile_order=1, overwrite=True, **kw)


def _robust_keep(sc, ref, views):
    """Pixels of the listed views (concatenated) that carry a loss gradient on
    both sides: unflagged by the oracle and with an L1 sign that no rounding
    can flip."""
    offs = sc.pixel_offsets
    sel = np.concatenate([np.arange(offs[v], offs[v] + sc.view_pixels(v)) for v in views])
    near = np.any(np.abs(ref["rgb"] - sc.target_rgb[:, sel]) < 5e-4, axis=0)
    if sc.target_depth is not None and sc.w_depth != 0.0:
        near |= np.abs(ref["depth"] - sc.target_depth[sel]) < 5e-4
    return sel, ~(ref["flags"] | near)


def _fused_masked(rast, gs, params, mask):
    out, ws = rast.forward(gs, params)
    ws = rast.workspace(gs, params, max_pairs=ws.n_pairs + 4096)
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    for g in grads:           # overwrite mode: nothing needs clearing
        for t in g.values():
            t.fill_(13.0)
    dvm.fill_(13.0)
    loss = torch.full((1,), 13.0, device="cuda")
    rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss, mask=mask)
    torch.cuda.synchronize()
    assert rast.query(gs, ws)[0] == 0
    return out, grads, dvm, float(loss), ws


def _compare_grads(tag, grads, dvm, rg, rdvm, submaps, views):
    worst = (0.0, 0.0)
    for s in submaps:
        for k in PLANES:
            e = grad_errors(to_np(grads[s][k]), rg[s][k])
            worst = (max(worst[0], e[0]), max(worst[1], e[1]))
            assert_grad_close(to_np(grads[s][k]), rg[s][k], f"{tag}[{s}].{k}")
    d = to_np(dvm)
    e = grad_errors(d[views], rdvm[views])
    assert_grad_close(d[views], rdvm[views], f"{tag}.viewmat")
    _say(f"PARITY {tag}: surfel gradients worst rel L2 {worst[0]:.2e}, worst element {worst[1]:.2e}; "
         f"pose rel L2 {e[0]:.2e}, worst element {e[1]:.2e}")
    return worst, e


def _fused_vs_oracle(rast, sc, views, tag, params=None, okw=None):
    """params: one raster-parameter set or a list of them (launches), each
    run on the GPU against the same oracle forward and backward."""
    okw = okw or {}
    gs = GpuScene.from_scene(sc)
    _say(f"{tag}: oracle forward of views {views}")
    ref = oracle.render_scene(sc, views=views, **okw)
    sel, keep = _robust_keep(sc, ref, views)
    assert keep.mean() > 0.98, keep.mean()
    mask = np.zeros(sc.total_pixels, np.uint8)
    mask[sel] = keep
    L, g = oracle.l1_loss(sc, ref, views=views, mask=keep)
    _say(f"{tag}: oracle backward")
    rg, rdvm = oracle.backward_scene(sc, g, views=views, **okw)
    used = sorted({sc.views[v][2] for v in views})
    plist = params if isinstance(params, list) else [params or _bench_params(rast)]
    res = []
    for p in plist:
        t = (f"{tag} {p.tile_w}x{p.tile_h}/order {p.tile_order}/waves {p.tile_waves}/depth {p.lds_depth}"
             + ("/deterministic" if p.deterministic else ""))
        _say(f"{t}: fused batch of {gs.n_views} views")
        out, grads, dvm, loss, ws = _fused_masked(rast, gs, p, torch.from_numpy(mask).cuda())
        got = {k: x[..., torch.from_numpy(sel).cuda()] for k, x in out.items()}
        assert_images_close(got, ref, ~ref["flags"], what=t)
        assert abs(loss - L) <= 2e-5 * max(L, 1e-6), (loss, L)
        res.append(_compare_grads(t, grads, dvm, rg, rdvm, used, views))
        # views without loss pixels store a zero pose gradient
        others = [v for v in range(sc.n_views) if v not in views]
        if others:
            assert float(dvm[others].abs().max()) == 0.0
    return res if isinstance(params, list) else res[0]


def test_fused_headline_views_match_oracle(rast):
    """Headline batch (16 x 640x480, 300k surfels): views 0 and 9 carry the
    loss; surfel and pose gradients of the timed kernel against the oracle,
    and of the same launch with deterministic sums."""
    _fused_vs_oracle(rast, scenes.headline(), [0, 9], "headline v0,v9",
                     params=[_bench_params(rast), _bench_params(rast, deterministic=True)])


def test_fused_config1_matches_oracle(rast):
    """Config 1 (one 640x480 view, 300k surfels) at 16x16 and at the launches
    the autotuner picks for it: 16x8 tiles with one wave per 8x8 block, and
    8x8 tiles at LDS depth 64 and 32."""
    _fused_vs_oracle(rast, scenes.config1(), [0], "config1",
                     params=[_bench_params(rast),
                             rast.params(tile=(16, 8), tile_order=1, tile_waves=2, overwrite=True),
                             rast.params(tile=(8, 8), tile_order=1, overwrite=True),
                             rast.params(tile=(8, 8), tile_order=1, lds_depth=32, overwrite=True)])


def test_fused_config2_view_matches_oracle(rast):
    """Config 2 (16 x 512x384 over 1M shared surfels): view 3, at 16x16 and at
    the autotuner's picks for this batch (16x16 and 32x32 in image order)."""
    _fused_vs_oracle(rast, scenes.config2(), [3], "config2 v3",
                     params=[_bench_params(rast), rast.params(tile=(16, 16), tile_order=2, overwrite=True),
                             rast.params(tile=(32, 32), tile_order=2, overwrite=True)])


def test_fused_config3_views_match_oracle(rast):
    """Config 3 (64 uneven views over 8 submaps): its largest 1280x720 view and
    a 320x240 view of another submap, with pose gradients; at the benchmark's
    16x16 launch and at the 32x32 launch the autotuner picks for this batch
    (the per-config block of the benchmark times both)."""
    sc = scenes.config3()
    big = max(range(sc.n_views), key=lambda v: sc.views[v][0] * sc.views[v][1])
    small = next(v for v in range(sc.n_views)
                 if sc.views[v][:2] == (320, 240) and sc.views[v][2] != sc.views[big][2])
    _fused_vs_oracle(rast, sc, [small, big], f"config3 v{small},v{big}",
                     params=[_bench_params(rast), rast.params(tile=(32, 32), tile_order=1, overwrite=True)])


def test_fused_config4_views_match_oracle(rast):
    """Config 4 (32 per-pixel maps of 518x392, each view rendering its own
    frame): views 5 and 20 carry the loss; at 16x16 and at the autotuner's
    16x8 launch with LDS depth 32."""
    _fused_vs_oracle(rast, scenes.config4(), [5, 20], "config4 v5,v20",
                     params=[_bench_params(rast),
                             rast.params(tile=(16, 8), tile_order=1, lds_depth=32, overwrite=True)])


# ------------------------------------------------------------ edge parameters
EDGE = dict(bg=(0.2, 0.1, 0.3), alpha_max=0.999, t_min=1e-3, rho_max=2.5, near=1.0)


def _edge_scene():
    """Small scene for non-default parameters: centres from z = 0.5 (some in
    front of the near plane at 1.0), a tenth of the surfels fully opaque (the
    0.999 clamp is active at their centres), depth targets."""
    sc = scenes.random_scene(61, 5000, 96, 72, n_views=2, lo=(-1, -1, 0.5), hi=(1, 1, 6),
                             scale_lo=0.03, scale_hi=0.2)
    op = sc.submaps[0]["opacity"]
    op[::10] = 1.0
    return sc


def test_edge_parameters_fused(rast):
    sc = _edge_scene()
    okw = dict(EDGE)
    _fused_vs_oracle(rast, sc, [0, 1], "edge params fused", params=_bench_params(rast, **EDGE), okw=okw)


def test_edge_parameters_backward(rast):
    """fm_backward with every output plane carrying a random upstream
    gradient, under the same non-default parameters."""
    sc = _edge_scene()
    gs = GpuScene.from_scene(sc)
    p = rast.params(**EDGE)
    out, ws = rast.forward(gs, p)
    ref = oracle.render_scene(sc, **EDGE)
    keep = ~ref["flags"]
    assert keep.mean() > 0.98
    assert_images_close(out, ref, keep, what="edge forward")
    g = random_upstream(np.random.default_rng(62), gs.npx, keep)
    gt = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in g.items()}
    grads, dvm = gs.zero_grads()
    rast.backward(gs, ws, out, gt, grads, dvm)
    torch.cuda.synchronize()
    rg, rdvm = oracle.backward_scene(sc, g, **EDGE)
    _compare_grads("edge params backward", grads, dvm, rg, rdvm, [0], [0, 1])


# ------------------------------------------------------ chunked descriptors
def _many_submaps_scene():
    """20 views over 9 small submaps (more than the 16 views / 8 submaps one
    descriptor launch carries, so the chunked descriptor path runs)."""
    base = [scenes.random_scene(70 + i, 600 + 150 * i, 48, 40, scale_lo=0.03, scale_hi=0.15)
            for i in range(9)]
    views = [(48, 40, j % 9) for j in range(20)]
    rng = np.random.default_rng(71)
    intr = np.concatenate([base[s].intr for (_, _, s) in views])
    vm = np.concatenate([base[s].viewmat for (_, _, s) in views]).copy()
    vm[:, [3, 7]] += rng.uniform(-0.1, 0.1, (len(views), 2)).astype(np.float32)
    sc = scenes.Scene("many_submaps", [b.submaps[0] for b in base], views, intr, vm, w_rgb=1.0, w_depth=0.1)
    r = np.random.default_rng(72)
    sc.target_rgb = r.random((3, sc.total_pixels)).astype(np.float32)
    sc.target_depth = r.uniform(1.0, 8.0, sc.total_pixels).astype(np.float32)
    return sc


def test_chunked_batch_fused_matches_oracle(rast):
    sc = _many_submaps_scene()
    _fused_vs_oracle(rast, sc, list(range(sc.n_views)), "20 views / 9 submaps fused")


def test_chunked_batch_backward_matches_oracle(rast):
    sc = _many_submaps_scene()
    gs = GpuScene.from_scene(sc)
    out, ws = rast.forward(gs)
    ref = oracle.render_scene(sc)
    keep = ~ref["flags"]
    assert_images_close(out, ref, keep, what="20 views / 9 submaps")
    g = random_upstream(np.random.default_rng(73), gs.npx, keep)
    gt = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in g.items()}
    grads, dvm = gs.zero_grads()
    rast.backward(gs, ws, out, gt, grads, dvm)
    torch.cuda.synchronize()
    rg, rdvm = oracle.backward_scene(sc, g)
    _compare_grads("20 views / 9 submaps backward", grads, dvm, rg, rdvm, list(range(9)),
                   list(range(sc.n_views)))
