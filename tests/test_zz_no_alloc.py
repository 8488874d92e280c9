"""fm_fwd_bwd_l1_noalloc (the fused call on the library's static scratch
array) against fm_fwd_bwd_l1 on a caller workspace, through the C ABI: two
calls in a row, the second on a smaller batch, so stale scratch contents of
the first call must not leak into the second."""
import numpy as np
import pytest
import torch

from paper_2604_03092_amd import native, scenes
from paper_2604_03092_amd.raster import GpuScene, Rasterizer
from tests.gpu_util import assert_grad_close, to_np

pytestmark = pytest.mark.gpu

PLANES = ("mean", "quat", "scale", "opacity", "color")


@pytest.fixture(scope="module")
def rast():
    return Rasterizer()


def _run_both(rast, gs, params, max_pairs):
    """(reference results, no-alloc results, pair status) of one batch."""
    res = []
    for kind in ("ws", "noalloc"):
        out = rast.new_outputs(gs)
        grads, dvm = gs.zero_grads()
        loss = torch.zeros(1, device="cuda")
        if kind == "ws":
            ws = rast.workspace(gs, params, max_pairs=max_pairs)
            rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss)
            torch.cuda.synchronize()
            st, n, req = rast.query(gs, ws)
            assert st == 0
        else:
            status = torch.full((2,), -7, dtype=torch.int64, device="cuda")
            rast.fwd_bwd_l1_noalloc(gs, params, max_pairs, out, grads, dvm, loss, pair_status=status)
            torch.cuda.synchronize()
            got = status.cpu().numpy()
            assert got[0] == req and got[1] == 0, (got, req)
        res.append((out, grads, dvm, float(loss)))
    return res


def _compare(tag, a, b, bitwise):
    (oa, ga, da, la), (ob, gb, db, lb) = a, b
    for k in oa:
        assert torch.equal(oa[k], ob[k]), f"{tag}: {k} differs"
    if bitwise:
        assert la == lb, (tag, la, lb)
        for s in range(len(ga)):
            for k in PLANES:
                assert torch.equal(ga[s][k], gb[s][k]), f"{tag}: grad {k} differs"
        assert torch.equal(da, db)
        return
    assert abs(la - lb) <= 1e-6 * max(abs(la), 1e-6), (tag, la, lb)
    for s in range(len(ga)):
        for k in PLANES:
            assert_grad_close(to_np(gb[s][k]), to_np(ga[s][k]), f"{tag}.{k}")
    assert_grad_close(to_np(db), to_np(da), f"{tag}.viewmat")


def test_noalloc_matches_workspace_call_twice(rast):
    # first call: one 640x480 view of 300k surfels (the largest single view)
    big = GpuScene.from_scene(scenes.config1())
    p = rast.params(tile=(16, 16))
    _, ws = rast.forward(big, p)
    max_pairs = ws.n_pairs + 4096
    assert rast.workspace_size(big, p, max_pairs) <= native.FM_NOALLOC_SCRATCH_BYTES
    # the documented limit: this view fits with room for 1.5M pairs
    assert rast.workspace_size(big, p, 1_500_000) <= native.FM_NOALLOC_SCRATCH_BYTES
    del ws
    print("no-alloc: 640x480 / 300k", flush=True)
    a, b = _run_both(rast, big, p, max_pairs)
    _compare("640x480/300k", a, b, bitwise=False)
    # second call, smaller: the 64x48 / 2k scene, deterministic sums (bitwise)
    small = GpuScene.from_scene(scenes.config0())
    pd = rast.params(tile=(16, 16), deterministic=True)
    print("no-alloc: 64x48 / 2k deterministic", flush=True)
    a, b = _run_both(rast, small, pd, 1 << 14)
    _compare("64x48/2k det", a, b, bitwise=True)
    # and the small scene in the default mode
    a, b = _run_both(rast, small, p, 1 << 14)
    _compare("64x48/2k", a, b, bitwise=False)


def test_noalloc_rejects_batches_beyond_the_scratch(rast):
    gs = GpuScene.from_scene(scenes.headline())
    p = rast.params(tile=(16, 16))
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    loss = torch.zeros(1, device="cuda")
    with pytest.raises(native.FmError) as e:
        rast.fwd_bwd_l1_noalloc(gs, p, 16 << 20, out, grads, dvm, loss)
    assert e.value.status == native.FM_ERR_WORKSPACE
    assert "static scratch" in str(e.value)
