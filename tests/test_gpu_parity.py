"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Every test seeds its inputs with the scene generators; the oracle sees the
same float32 arrays.  Output planes are compared on pixels the oracle does
not flag; upstream gradients are zeroed on flagged pixels on both sides."""
import numpy as np
import pytest
import torch

import oracle
from paper_2604_03092_amd import scenes
from paper_2604_03092_amd.raster import GpuScene, Rasterizer
from tests.gpu_util import (assert_grad_close, assert_images_close, assert_pairs_match, random_upstream,
                            to_np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rast():
    return Rasterizer()


def _say(msg):
    print(msg, flush=True)


def _oracle_forward(sc, views=None, **kw):
    return oracle.render_scene(sc, views=views, **kw)


def _gpu_pairs_by_view(rast, gs, ws, sc, tile):
    tile_ids, surf, view, ts, te = rast.debug_pairs(gs, ws)
    return tile_ids, surf, view, ts, te


# ------------------------------------------------------------------ forward
@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (16, 8), (32, 8), (32, 32)])
def test_config0_forward_and_pairs(rast, tile):
    sc = scenes.config0()
    _say(f"config0 forward tile={tile}")
    gs = GpuScene.from_scene(sc)
    p = rast.params(tile=tile)
    out, ws = rast.forward(gs, p)
    torch.cuda.synchronize()
    ref = _oracle_forward(sc)
    keep = ~ref["flags"]
    assert keep.mean() > 0.99
    assert_images_close(out, ref, keep, what="config0")
    # pair list and tile ranges: bit-exact
    b = oracle.bin_view(sc.submaps[0], 64, 48, sc.intr[0], sc.viewmat[0], tile_w=tile[0], tile_h=tile[1])
    t, s, v, ts, te = rast.debug_pairs(gs, ws)
    kept = assert_pairs_match(b, t, s, ts, te)
    _say(f"config0 tile={tile}: {kept:.3f} of the oracle's pairs kept")
    starts = np.concatenate([[0], np.cumsum(te - ts)[:-1]])
    assert np.array_equal(ts[te > ts], starts[te > ts])


def test_tile_shape_does_not_change_images(rast):
    """Images are bitwise the same for every tile shape and both tile orders."""
    sc = scenes.random_scene(5, 20000, 200, 136, scale_lo=0.02, scale_hi=0.15)
    gs = GpuScene.from_scene(sc)
    ref = None
    for tile, order, waves in [((16, 16), 1, 1), ((16, 16), 2, 1), ((8, 8), 1, 1), ((16, 8), 2, 1),
                               ((32, 8), 1, 1), ((32, 32), 1, 1), ((32, 32), 2, 1), ((16, 16), 1, 2),
                               ((16, 8), 2, 2), ((32, 8), 1, 2)]:
        _say(f"tile invariance {tile} order {order} waves {waves}")
        out, _ = rast.forward(gs, rast.params(tile=tile, tile_order=order, tile_waves=waves))
        got = {k: v.cpu().numpy() for k, v in out.items()}
        if ref is None:
            ref = got
        else:
            for k in ref:
                assert np.array_equal(got[k], ref[k]), (tile, k)


# ------------------------------------------------------------------ backward
@pytest.mark.parametrize("name,seed,tile", [("config0", 1, (16, 16)), ("dense", 2, (16, 16)),
                                           ("dense", 3, (32, 32)), ("dense", 4, (8, 8))])
def test_backward_small(rast, name, seed, tile):
    sc = scenes.config0() if name == "config0" else scenes.random_scene(
        33, 4000, 72, 56, scale_lo=0.03, scale_hi=0.2)
    _say(f"backward {name} tile={tile}")
    gs = GpuScene.from_scene(sc)
    out, ws = rast.forward(gs, rast.params(tile=tile))
    ref = _oracle_forward(sc)
    keep = ~ref["flags"]
    rng = np.random.default_rng(seed)
    g = random_upstream(rng, gs.npx, keep)
    gt = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in g.items()}
    grads, dvm = gs.zero_grads()
    rast.backward(gs, ws, out, gt, grads, dvm)
    torch.cuda.synchronize()
    rg, rdvm = oracle.backward_scene(sc, g)
    for k in ("mean", "quat", "scale", "opacity", "color"):
        assert_grad_close(to_np(grads[0][k]), rg[0][k], f"{name}.{k}")
    assert_grad_close(to_np(dvm), rdvm, f"{name}.viewmat")


@pytest.mark.parametrize("tile", [(16, 16), (32, 32)])
def test_fused_l1_config0(rast, tile):
    sc = scenes.config0()
    _say(f"fused l1 config0 tile={tile}")
    gs = GpuScene.from_scene(sc)
    ref = _oracle_forward(sc)
    # pixels whose L1 sign is not decided robustly are masked on both sides
    near = np.any(np.abs(ref["rgb"] - sc.target_rgb) < 5e-4, axis=0)
    keep = ~(ref["flags"] | near)
    mask = torch.from_numpy(keep.astype(np.uint8)).cuda()
    ws = rast.workspace(gs, rast.params(tile=tile))
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    loss = torch.zeros(1, device="cuda")
    rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss, mask=mask)
    torch.cuda.synchronize()
    assert rast.query(gs, ws)[0] == 0
    L, g = oracle.l1_loss(sc, ref, mask=keep)
    assert abs(float(loss) - L) <= 1e-5 * max(1.0, abs(L))
    assert_images_close(out, ref, keep, what="fused")
    rg, rdvm = oracle.backward_scene(sc, g)
    for k in ("mean", "quat", "scale", "opacity", "color"):
        assert_grad_close(to_np(grads[0][k]), rg[0][k], f"fused.{k}")
    assert_grad_close(to_np(dvm), rdvm, "fused.viewmat")


@pytest.mark.parametrize("tile,waves,depth,det", [((16, 16), 2, 32, False), ((32, 8), 2, 128, False),
                                                  ((16, 8), 2, 64, True), ((16, 16), 1, 128, False),
                                                  ((32, 32), 1, 32, False)])
def test_work_split_and_lds_depth_match_oracle(rast, tile, waves, depth, det):
    """The fused call with one wave per 8x8 block and other LDS batch depths
    against the oracle (three views over two submaps, depth loss)."""
    sc = scenes.random_scene(43, 6000, 96, 72, n_views=3, scale_lo=0.03, scale_hi=0.2)
    _say(f"work split tile={tile} waves={waves} depth={depth} det={det}")
    gs = GpuScene.from_scene(sc)
    ref = _oracle_forward(sc)
    near = np.any(np.abs(ref["rgb"] - sc.target_rgb) < 5e-4, axis=0) | (np.abs(ref["depth"] - sc.target_depth) < 5e-4)
    keep = ~(ref["flags"] | near)
    mask = torch.from_numpy(keep.astype(np.uint8)).cuda()
    p = rast.params(tile=tile, tile_waves=waves, lds_depth=depth, deterministic=det)
    _, ws = rast.forward(gs, p)
    ws = rast.workspace(gs, p, max_pairs=ws.n_pairs + 4096)
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    loss = torch.zeros(1, device="cuda")
    rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss, mask=mask)
    torch.cuda.synchronize()
    assert rast.query(gs, ws)[0] == 0
    L, g = oracle.l1_loss(sc, ref, mask=keep)
    assert abs(float(loss) - L) <= 1e-5 * max(1.0, abs(L))
    assert_images_close(out, ref, ~ref["flags"], what="split")
    rg, rdvm = oracle.backward_scene(sc, g)
    for k in ("mean", "quat", "scale", "opacity", "color"):
        assert_grad_close(to_np(grads[0][k]), rg[0][k], f"split.{k}")
    assert_grad_close(to_np(dvm), rdvm, "split.viewmat")
    # the backward through fm_backward with the same split
    gu = random_upstream(np.random.default_rng(44), gs.npx, ~ref["flags"])
    gt = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in gu.items()}
    out2, ws2 = rast.forward(gs, rast.params(tile=tile, tile_waves=waves, deterministic=det))
    grads2, dvm2 = gs.zero_grads()
    rast.backward(gs, ws2, out2, gt, grads2, dvm2)
    torch.cuda.synchronize()
    rg2, rdvm2 = oracle.backward_scene(sc, gu)
    for k in ("mean", "quat", "scale", "opacity", "color"):
        assert_grad_close(to_np(grads2[0][k]), rg2[0][k], f"split bwd.{k}")
    assert_grad_close(to_np(dvm2), rdvm2, "split bwd.viewmat")


def test_invalid_work_split(rast):
    sc = scenes.config0()
    gs = GpuScene.from_scene(sc)
    from paper_2604_03092_amd import native
    for kw in (dict(tile_waves=3), dict(lds_depth=48), dict(deterministic=True, lds_depth=32)):
        with pytest.raises(native.FmError) as e:
            rast.forward(gs, rast.params(**kw))
        assert e.value.status == native.FM_ERR_INVALID_ARG, kw


# ------------------------------------------------------- deterministic mode
def _fused_run(rast, gs, ws):
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    loss = torch.zeros(1, device="cuda")
    rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss)
    torch.cuda.synchronize()
    assert rast.query(gs, ws)[0] == 0
    flat = {f"{s}.{k}": to_np(v) for s, g in enumerate(grads) for k, v in g.items()}
    flat["viewmat"] = to_np(dvm)
    return {k: v.cpu().numpy() for k, v in out.items()}, float(loss), flat


@pytest.mark.parametrize("tile", [(16, 16), (32, 32)])
def test_deterministic_fused_is_reproducible(rast, tile):
    """Three views over two submaps with heavy overlap (many tiles add into
    one entry).  Deterministic mode: two fused steps agree bitwise in loss,
    surfel and pose gradients; images equal the default mode's bitwise and
    gradients agree with it to rounding."""
    sc = scenes.random_scene(21, 12000, 96, 72, n_views=3, scale_lo=0.05, scale_hi=0.3)
    sc.submaps.append({k: np.ascontiguousarray(v[..., ::2]) for k, v in sc.submaps[0].items()})
    sc.views[1] = (sc.views[1][0], sc.views[1][1], 1)
    gs = GpuScene.from_scene(sc)
    _say(f"deterministic fused tile={tile}")
    ws_d = rast.workspace(gs, rast.params(tile=tile, deterministic=True), max_pairs=400_000)
    ws_n = rast.workspace(gs, rast.params(tile=tile), max_pairs=400_000)
    # the same sums in image tile order: the deterministic result does not
    # depend on the order in which tiles run
    ws_i = rast.workspace(gs, rast.params(tile=tile, deterministic=True, tile_order=2), max_pairs=400_000)
    img_d, loss_d, g_d = _fused_run(rast, gs, ws_d)
    img_d2, loss_d2, g_d2 = _fused_run(rast, gs, ws_d)
    img_i, loss_i, g_i = _fused_run(rast, gs, ws_i)
    img_n, loss_n, g_n = _fused_run(rast, gs, ws_n)
    assert loss_d == loss_d2
    for k in g_d:
        assert np.array_equal(g_d[k], g_d2[k]), k
        assert np.array_equal(g_d[k], g_i[k]), k
        assert_grad_close(g_d[k], g_n[k], f"det-vs-atomic {k}", rel=1e-4)
    for k in img_d:
        assert np.array_equal(img_d[k], img_d2[k]), k
        assert np.array_equal(img_d[k], img_n[k]), k
        assert np.array_equal(img_d[k], img_i[k]), k
    assert loss_d == loss_n


@pytest.mark.parametrize("tile", [(16, 16), (32, 32)])
def test_deterministic_backward_with_normals_matches_oracle(rast, tile):
    """fm_backward in deterministic mode with every output plane carrying a
    gradient (20-float slots): reproducible and equal to the oracle's
    gradients within the usual tolerance; pairs as in the default mode."""
    sc = scenes.random_scene(33, 4000, 72, 56, scale_lo=0.03, scale_hi=0.2)
    gs = GpuScene.from_scene(sc)
    _say(f"deterministic backward tile={tile}")
    p = rast.params(tile=tile, deterministic=True)
    out, ws = rast.forward(gs, p)
    ref = _oracle_forward(sc)
    keep = ~ref["flags"]
    assert_images_close(out, ref, keep, what="deterministic")
    out_n, ws_n = rast.forward(gs, rast.params(tile=tile))
    pairs_d, pairs_n = rast.debug_pairs(gs, ws), rast.debug_pairs(gs, ws_n)
    for a, b in zip(pairs_d, pairs_n):
        assert np.array_equal(a, b)
    g = random_upstream(np.random.default_rng(5), gs.npx, keep)
    gt = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in g.items()}
    runs = []
    for _ in range(2):
        grads, dvm = gs.zero_grads()
        rast.backward(gs, ws, out, gt, grads, dvm)
        torch.cuda.synchronize()
        runs.append(({k: to_np(v) for k, v in grads[0].items()}, to_np(dvm)))
    rg, rdvm = oracle.backward_scene(sc, g)
    for k in ("mean", "quat", "scale", "opacity", "color"):
        assert np.array_equal(runs[0][0][k], runs[1][0][k]), k
        assert_grad_close(runs[0][0][k], rg[0][k], f"deterministic.{k}")
    assert np.array_equal(runs[0][1], runs[1][1])
    assert_grad_close(runs[0][1], rdvm, "deterministic.viewmat")


def test_backward_in_the_other_tile_order(rast):
    """A forward in image order followed by backwards in either order on the
    same workspace: the tile order only schedules, so the deterministic
    gradients are the same bits."""
    from paper_2604_03092_amd.raster import Workspace
    sc = scenes.random_scene(34, 4000, 72, 56, scale_lo=0.03, scale_hi=0.2)
    gs = GpuScene.from_scene(sc)
    _say("backward in the other tile order")
    out, ws = rast.forward(gs, rast.params(tile_order=2, deterministic=True))
    keep = ~_oracle_forward(sc)["flags"]
    g = random_upstream(np.random.default_rng(6), gs.npx, keep)
    gt = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in g.items()}
    res = []
    for order in (2, 1):
        w = Workspace(ws.buf, ws.nbytes, ws.max_pairs, rast.params(tile_order=order, deterministic=True))
        grads, dvm = gs.zero_grads()
        rast.backward(gs, w, out, gt, grads, dvm)
        torch.cuda.synchronize()
        res.append(({k: to_np(v) for k, v in grads[0].items()}, to_np(dvm)))
    for k in res[0][0]:
        assert np.array_equal(res[0][0][k], res[1][0][k]), k
    assert np.array_equal(res[0][1], res[1][1])


def test_overwrite_stores_gradients(rast):
    """overwrite = 1: the fused call and fm_backward store surfel gradients,
    pose gradients and the loss over whatever the buffers held, equal bitwise
    to accumulating into zeroed buffers; a submap no view renders keeps its
    contents."""
    sc = scenes.random_scene(23, 6000, 80, 60, n_views=2, scale_lo=0.03, scale_hi=0.2)
    sc.submaps.append({k: np.ascontiguousarray(v[..., :500]) for k, v in sc.submaps[0].items()})
    gs = GpuScene.from_scene(sc)
    _say("overwrite mode")
    res = {}
    for ow in (False, True):
        # (deterministic sums, so that the two modes can be compared bitwise)
        ws = rast.workspace(gs, rast.params(overwrite=ow, deterministic=True), max_pairs=200_000)
        out = rast.new_outputs(gs)
        grads, dvm = gs.zero_grads()
        loss = torch.zeros(1, device="cuda")
        if ow:
            for g in grads:
                for t in g.values():
                    t.fill_(7.0)
            dvm.fill_(7.0)
            loss.fill_(7.0)
        rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss)
        torch.cuda.synchronize()
        assert rast.query(gs, ws)[0] == 0
        res[ow] = ({k: to_np(v) for k, v in grads[0].items()}, to_np(dvm), float(loss),
                   {k: to_np(v) for k, v in grads[1].items()})
        up = {k: torch.ones_like(v) for k, v in out.items()}
        for g in grads:
            for t in g.values():
                t.fill_(3.0 if ow else 0.0)
        dvm.fill_(3.0 if ow else 0.0)
        rast.backward(gs, ws, out, up, grads, dvm)
        torch.cuda.synchronize()
        res[ow] += ({k: to_np(v) for k, v in grads[0].items()}, to_np(dvm))
    for k in res[False][0]:
        assert np.array_equal(res[True][0][k], res[False][0][k]), k
        assert np.array_equal(res[True][4][k], res[False][4][k]), k
        assert np.all(res[True][3][k] == 7.0), k  # submap 1 has no view
    assert np.array_equal(res[True][1], res[False][1])
    assert np.array_equal(res[True][5], res[False][5])
    assert res[True][2] == res[False][2]


# ------------------------------------------------------------------ batches
def test_batch_equals_single_views(rast):
    sc = scenes.random_scene(9, 30000, 160, 120, n_views=4, scale_lo=0.02, scale_hi=0.12)
    gs = GpuScene.from_scene(sc)
    _say("batch of 4 views")
    out, ws = rast.forward(gs)
    rng = np.random.default_rng(3)
    g = random_upstream(rng, gs.npx, np.ones(gs.npx, bool))
    gt = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in g.items()}
    grads, dvm = gs.zero_grads()
    rast.backward(gs, ws, out, gt, grads, dvm)
    acc_grads, _ = gs.zero_grads()
    for v in range(4):
        gv = GpuScene(gs.submaps, [gs.views[v]], gs.intr[v:v + 1].contiguous(), gs.viewmat[v:v + 1].contiguous())
        o1, w1 = rast.forward(gv)
        sl = slice(gs.pixel_offsets[v], gs.pixel_offsets[v] + gv.npx)
        for k in out:
            assert torch.equal(o1[k], out[k][..., sl]), (v, k)
        g1 = {k: x[..., sl].contiguous() for k, x in gt.items()}
        d1 = torch.zeros(1, 12, device="cuda")
        rast.backward(gv, w1, o1, g1, acc_grads, d1)
        assert torch.allclose(d1[0], dvm[v], rtol=1e-4, atol=1e-6 * float(dvm.abs().max()))
    for k in acc_grads[0]:
        assert_grad_close(to_np(grads[0][k]), to_np(acc_grads[0][k]), f"batch.{k}", rel=1e-5)


def test_multi_submap_batch(rast):
    base = [scenes.random_scene(40 + i, 3000 * (i + 1), 64, 48, scale_lo=0.03, scale_hi=0.15) for i in range(3)]
    views = [(64, 48, 0), (64, 48, 2), (64, 48, 1), (64, 48, 2)]
    intr = np.concatenate([base[s].intr for (_, _, s) in views])
    vm = np.concatenate([base[s].viewmat for (_, _, s) in views])
    sc = scenes.Scene("multi", [b.submaps[0] for b in base], views, intr, vm)
    _say("multi-submap batch")
    gs = GpuScene.from_scene(sc)
    out, ws = rast.forward(gs)
    ref = _oracle_forward(sc)
    keep = ~ref["flags"]
    assert_images_close(out, ref, keep, what="multi")
    rng = np.random.default_rng(4)
    g = random_upstream(rng, gs.npx, keep)
    gt = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in g.items()}
    grads, dvm = gs.zero_grads()
    rast.backward(gs, ws, out, gt, grads, dvm)
    torch.cuda.synchronize()
    rg, rdvm = oracle.backward_scene(sc, g)
    for s in range(3):
        for k in ("mean", "quat", "scale", "opacity", "color"):
            assert_grad_close(to_np(grads[s][k]), rg[s][k], f"multi[{s}].{k}")
    assert_grad_close(to_np(dvm), rdvm, "multi.viewmat")


# ------------------------------------------------------------------ full size
def test_config1_forward_backward(rast):
    sc = scenes.config1()
    _say("config1 forward")
    gs = GpuScene.from_scene(sc)
    out, ws = rast.forward(gs)
    torch.cuda.synchronize()
    ref = _oracle_forward(sc)
    keep = ~ref["flags"]
    _say(f"config1 flagged fraction {1 - keep.mean():.2e}")
    assert keep.mean() > 0.99
    assert_images_close(out, ref, keep, what="config1")
    _say("config1 pairs")
    b = oracle.bin_view(sc.submaps[0], 640, 480, sc.intr[0], sc.viewmat[0])
    t, s, v, ts, te = rast.debug_pairs(gs, ws)
    kept = assert_pairs_match(b, t, s, ts, te)
    _say(f"config1: {kept:.3f} of the oracle's pairs kept")
    _say("config1 backward")
    near = np.any(np.abs(ref["rgb"] - sc.target_rgb) < 5e-4, axis=0) | (
        np.abs(ref["depth"] - sc.target_depth) < 5e-4)
    keep2 = keep & ~near
    L, g = oracle.l1_loss(sc, ref, mask=keep2)
    gt = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in g.items()}
    grads, dvm = gs.zero_grads()
    rast.backward(gs, ws, out, gt, grads, dvm)
    torch.cuda.synchronize()
    rg, rdvm = oracle.backward_scene(sc, g)
    for k in ("mean", "quat", "scale", "opacity", "color"):
        assert_grad_close(to_np(grads[0][k]), rg[0][k], f"config1.{k}")
    assert_grad_close(to_np(dvm), rdvm, "config1.viewmat")


# ------------------------------------------------------------------ edge cases
def test_capacity_overflow_then_retry(rast):
    sc = scenes.config0()
    gs = GpuScene.from_scene(sc)
    _say("capacity overflow")
    ws = rast.workspace(gs, max_pairs=100)
    out = rast.new_outputs(gs)
    rast.forward_into(gs, ws, out)
    st, n, req = rast.query(gs, ws)
    assert st == 2 and n == 100 and req > 100
    out2, ws2 = rast.forward(gs)            # grows and succeeds
    assert rast.query(gs, ws2)[0] == 0
    ref = _oracle_forward(sc)
    assert_images_close(out2, ref, ~ref["flags"], what="after grow")


def test_capacity_overflow_counts_every_pair(rast):
    """A 640x480 view of 300k surfels (about 90 blocks of the pair count
    scan) with room for half its pairs: the call reports the overflow, stores
    exactly the capacity, and the required count equals the pair count of a
    call with room for all of them."""
    gs = GpuScene.from_scene(scenes.config1())
    _say("capacity overflow, 640x480 / 300k")
    out, ws = rast.forward(gs)
    torch.cuda.synchronize()
    st, n_full, req_full = rast.query(gs, ws)
    assert st == 0 and n_full == req_full > 100_000
    cap = req_full // 2
    ws2 = rast.workspace(gs, max_pairs=cap)
    rast.forward_into(gs, ws2, rast.new_outputs(gs))
    torch.cuda.synchronize()
    st2, n2, req2 = rast.query(gs, ws2)
    assert st2 == 2 and n2 == cap and req2 == req_full


def test_empty_and_culled(rast):
    # every surfel culled: NaN, zero quaternion, behind the camera, transparent
    n = 8
    sm = dict(mean=np.tile(np.array([[0.0], [0.0], [3.0]], np.float32), (1, n)),
              quat=np.tile(np.array([[1.0], [0.0], [0.0], [0.0]], np.float32), (1, n)),
              scale=np.full((2, n), 0.3, np.float32), opacity=np.full(n, 0.8, np.float32),
              color=np.ones((3, n), np.float32))
    sm["mean"][0, 0] = np.nan
    sm["quat"][:, 1] = 0.0
    sm["mean"][2, 2] = -1.0
    sm["opacity"][3] = 0.001
    sm["scale"][1, 4] = 0.0
    sm["quat"][2, 5] = np.inf
    sm["mean"][2, 6] = 0.1
    sm["color"][1, 7] = np.nan
    sc = scenes.Scene("culled", [sm], [(32, 24, 0)], np.array([[30, 30, 16, 12]], np.float32),
                      np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32))
    gs = GpuScene.from_scene(sc)
    _say("all culled")
    out, ws = rast.forward(gs)
    assert float(out["alpha"].abs().max()) == 0.0 and float(out["rgb"].abs().max()) == 0.0
    assert rast.query(gs, ws)[1] == 0
    g = {k: torch.ones_like(v) for k, v in out.items()}
    grads, dvm = gs.zero_grads()
    rast.backward(gs, ws, out, g, grads, dvm)
    for k in grads[0]:
        assert float(grads[0][k].abs().max()) == 0.0
    # empty submap
    sm0 = {k: v[..., :0].copy() for k, v in sm.items()}
    gs0 = GpuScene.from_scene(scenes.Scene("empty", [sm0], [(20, 10, 0)], sc.intr, sc.viewmat))
    out0, _ = rast.forward(gs0)
    assert float(out0["alpha"].abs().max()) == 0.0


def test_largest_view_crops_match_oracle(rast):
    """A 16384 x 16384 view (the largest accepted; 2^28 pixels, ~1M tiles, a
    three-pass tile sort) with two small surfel clusters in opposite corners:
    each cluster's crop equals the oracle's rendering of the same crop (a view
    with the principal point shifted by the crop corner) and every pixel
    outside the crops is exactly background."""
    sc = scenes.largest_view_clusters()
    gs = GpuScene.from_scene(sc)
    size, crop = sc.views[0][0], sc.meta["crop"]
    _say(f"largest view {size}x{size}")
    out, ws = rast.forward(gs)
    torch.cuda.synchronize()
    img = {k: v.view(-1, size, size) for k, v in out.items()}
    rest = {"alpha": img["alpha"].clone(), "rgb": img["rgb"][0].clone()}
    for (x0, y0) in sc.meta["crops"]:
        fx, fy, cx, cy = (float(x) for x in sc.intr[0])
        csc = scenes.Scene("crop", sc.submaps, [(crop, crop, 0)],
                           np.array([[fx, fy, cx - x0, cy - y0]], np.float32), sc.viewmat)
        ref = _oracle_forward(csc)
        keep = ~ref["flags"]
        assert keep.mean() > 0.99
        got = {k: v[:, y0:y0 + crop, x0:x0 + crop].reshape(v.shape[0], -1).squeeze(0) for k, v in img.items()}
        assert float(got["alpha"].max()) > 0.5  # the cluster is there
        assert_images_close(got, ref, keep, what=f"crop {x0},{y0}")
        for v in rest.values():
            v[..., y0:y0 + crop, x0:x0 + crop] = 0.0
    for k, v in rest.items():
        assert float(v.abs().max()) == 0.0, k


def test_invalid_arguments(rast):
    from paper_2604_03092_amd import native
    sc = scenes.config0()
    gs = GpuScene.from_scene(sc)
    with pytest.raises(native.FmError) as e:
        rast.workspace(gs, rast.params(tile=(12, 12)))
    assert e.value.status == native.FM_ERR_UNSUPPORTED
    for bad_params in (dict(alpha_max=1.5), dict(alpha_min=1e-7), dict(t_min=0.0), dict(t_min=1e-31)):
        with pytest.raises(native.FmError) as e:
            rast.workspace(gs, rast.params(**bad_params))
        assert e.value.status == native.FM_ERR_INVALID_ARG, bad_params
    for field, value in (("deterministic", 2), ("overwrite", -1), ("tile_order", 3)):
        p = rast.params()
        setattr(p, field, value)
        with pytest.raises(native.FmError) as e:
            rast.workspace(gs, p)
        assert e.value.status == native.FM_ERR_INVALID_ARG, field
    ws = rast.workspace(gs)
    ws.nbytes = 10
    with pytest.raises(native.FmError) as e:
        rast.forward_into(gs, ws, rast.new_outputs(gs))
    assert e.value.status == native.FM_ERR_WORKSPACE
    bad = GpuScene(gs.submaps, [(64, 48, 3)], gs.intr, gs.viewmat)
    with pytest.raises(native.FmError):
        rast.workspace(bad)


def test_autograd_matches_direct(rast):
    from paper_2604_03092_amd.raster import render
    sc = scenes.config0()
    gs = GpuScene.from_scene(sc)
    sub = {k: v.clone().requires_grad_(True) for k, v in gs.submaps[0].items()}
    vm = gs.viewmat.clone().requires_grad_(True)
    _say("autograd")
    rgb, depth, normal, alpha = render(rast, [sub], gs.views, gs.intr, vm)
    loss = (rgb * 0.3).sum() + (depth * 0.1).sum() + normal.sum() * 0.05 + alpha.sum() * 0.2
    loss.backward()
    out, ws = rast.forward(gs)
    g = dict(rgb=torch.full_like(out["rgb"], 0.3), depth=torch.full_like(out["depth"], 0.1),
             normal=torch.full_like(out["normal"], 0.05), alpha=torch.full_like(out["alpha"], 0.2))
    grads, dvm = gs.zero_grads()
    rast.backward(gs, ws, out, g, grads, dvm)
    for k in sub:
        assert_grad_close(to_np(sub[k].grad), to_np(grads[0][k]), f"autograd.{k}", rel=1e-5)
    assert_grad_close(to_np(vm.grad), to_np(dvm), "autograd.viewmat", rel=1e-5)


def test_overflowing_record_is_culled(rast):
    """A surfel whose plane coefficients would overflow FP32 (scale 1e25) is
    culled: the images equal those of the same scene with that surfel
    culled by its opacity instead, and every gradient stays finite."""
    import copy
    sc = scenes.config0()
    huge = copy.deepcopy(sc)
    sm = huge.submaps[0]
    sm["mean"][:, 0] = (0.0, 0.0, 3.0)
    sm["quat"][:, 0] = (1.0, 0.0, 0.0, 0.0)
    sm["scale"][:, 0] = (1e25, 1e25)
    gone = copy.deepcopy(huge)
    gone.submaps[0]["opacity"][0] = 1e-4  # below alpha_min: culled the ordinary way
    _say("overflowing record")
    res = []
    for s in (huge, gone):
        gs = GpuScene.from_scene(s)
        out, ws = rast.forward(gs)
        rng = np.random.default_rng(5)
        g = random_upstream(rng, gs.npx, np.ones(gs.npx, bool))
        gt = {k: torch.from_numpy(v.astype(np.float32)).cuda() for k, v in g.items()}
        grads, dvm = gs.zero_grads()
        rast.backward(gs, ws, out, gt, grads, dvm)
        torch.cuda.synchronize()
        res.append(({k: to_np(v) for k, v in out.items()}, {k: to_np(v) for k, v in grads[0].items()},
                    to_np(dvm)))
    (o1, g1, v1), (o2, g2, v2) = res
    for k in o1:
        assert np.array_equal(o1[k], o2[k]), k
    for k in g1:
        assert np.isfinite(g1[k]).all(), k
        assert np.all(g1[k][..., 0] == 0.0), k
        assert_grad_close(g1[k], g2[k], f"overflow.{k}")
    assert np.isfinite(v1).all()
    assert_grad_close(v1, v2, "overflow.viewmat")


def test_pixel_state_matches_oracle(rast):
    """Final transmittance and number of composited surfels per pixel."""
    sc = scenes.random_scene(12, 6000, 96, 64, scale_lo=0.03, scale_hi=0.2)
    gs = GpuScene.from_scene(sc)
    _say("pixel state")
    out, ws = rast.forward(gs)
    tf, nc = rast.pixel_state(gs, ws)
    ref = _oracle_forward(sc)
    keep = ~ref["flags"]
    assert np.array_equal(nc[keep], ref["n_contrib"][keep])
    assert np.abs(tf[keep] - ref["t_final"][keep]).max() <= 1e-5


def test_graph_replay_matches_eager(rast):
    """The fused call captured in a graph, replayed several times with eager
    work in between, reproduces the eager result every time."""
    sc = scenes.random_scene(13, 20000, 128, 96, n_views=3, scale_lo=0.02, scale_hi=0.12)
    gs = GpuScene.from_scene(sc)
    _say("graph replay")
    out0, ws = rast.forward(gs)
    ws = rast.workspace(gs, max_pairs=ws.n_pairs + 1024)
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    loss = torch.zeros(1, device="cuda")

    def step():
        for g in grads:
            for t in g.values():
                t.zero_()
        dvm.zero_()
        loss.zero_()
        rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss)

    step()
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in out.items()}
    ref_g = {k: v.clone() for k, v in grads[0].items()}
    ref_dvm, ref_loss = dvm.clone(), loss.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(4):
        out["rgb"].fill_(-1.0)
        grads[0]["mean"].fill_(123.0)
        graph.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(out[k], ref[k]), (rep, k)
        assert torch.allclose(loss, ref_loss, rtol=1e-6)
        for k in ref_g:
            assert torch.allclose(grads[0][k], ref_g[k], rtol=1e-4, atol=1e-6 * float(ref_g[k].abs().max())), (rep, k)
        assert torch.allclose(dvm, ref_dvm, rtol=1e-4, atol=1e-6 * float(ref_dvm.abs().max()))
        _ = torch.randn(1000, device="cuda").sum()   # eager work between replays


def test_graph_replay_deterministic_overwrite(rast):
    """Deterministic sums and stored gradients under graph capture: with no
    clearing in the graph and the buffers scribbled over between replays,
    every replay reproduces the eager result bitwise."""
    sc = scenes.random_scene(14, 20000, 128, 96, n_views=3, scale_lo=0.02, scale_hi=0.12)
    gs = GpuScene.from_scene(sc)
    _say("graph replay, deterministic + overwrite")
    p = rast.params(deterministic=True, overwrite=True)
    out0, ws = rast.forward(gs, p)
    ws = rast.workspace(gs, p, max_pairs=ws.n_pairs + 1024)
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    loss = torch.zeros(1, device="cuda")
    rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in out.items()}
    ref_g = {k: v.clone() for k, v in grads[0].items()}
    ref_dvm, ref_loss = dvm.clone(), loss.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss)
    for rep in range(4):
        out["rgb"].fill_(-1.0)
        for t in grads[0].values():
            t.fill_(123.0)
        dvm.fill_(5.0)
        loss.fill_(9.0)
        graph.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(out[k], ref[k]), (rep, k)
        for k in ref_g:
            assert torch.equal(grads[0][k], ref_g[k]), (rep, k)
        assert torch.equal(dvm, ref_dvm) and torch.equal(loss, ref_loss), rep
        _ = torch.randn(1000, device="cuda").sum()   # eager work between replays
