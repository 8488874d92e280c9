"""GPU parity of map fusion (fm_voxelize_fuse and fm_voxelize_fuse_batch through
the C ABI) against the FP64 fusion oracle: counts and order exact, values to
float32 rounding; a batch equals the concatenation of its frames."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import fusion
from paper_2604_03092_amd import native, scenes
from paper_2604_03092_amd.raster import PLANES, Fusion, FusionBatch, Rasterizer, _ptr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rast():
    return Rasterizer()


def _dev(planes):
    return {k: torch.from_numpy(np.ascontiguousarray(planes[k])).cuda() for k in PLANES}


def _tiny_frame(w, h, seed):
    rng = np.random.default_rng(seed)
    P = w * h
    q = rng.normal(size=(4, P))
    planes = dict(mean=np.stack([rng.uniform(-1, 1, P), rng.uniform(-1, 1, P), rng.uniform(2, 2.04, P)]),
                  quat=q / np.linalg.norm(q, axis=0), scale=rng.uniform(0.01, 0.1, (2, P)),
                  opacity=rng.uniform(0.3, 1, P), color=rng.random((3, P)))
    planes = {k: np.ascontiguousarray(v, np.float32) for k, v in planes.items()}
    return scenes.FusionFrame(w, h, planes, 1.05, np.array([0.9, 0.1, -0.3, 0.2], np.float32),
                              np.array([0.1, 0.2, -0.3], np.float32), rng.random(P).astype(np.float32))


def _check(fu, ref, n):
    for k in PLANES:
        want = ref[k].reshape(-1, n)
        got = fu.out[k].reshape(-1, fu.cap)[:, :n].cpu().numpy().astype(np.float64)
        tol = 2e-6 * (np.abs(want) + (1.0 if k == "mean" else 0.0) * 6.0) + 1e-7
        assert np.all(np.abs(got - want) <= tol), (k, np.max(np.abs(got - want) - tol))


@pytest.mark.parametrize("size", [(64, 48), (65, 47), (9, 7), (1, 1), (2, 1)])
@pytest.mark.parametrize("gate", [False, True])
def test_fusion_matches_oracle(rast, size, gate):
    w, h = size
    print(f"fusion {w}x{h} gate={gate}", flush=True)
    if w >= 3 and h >= 3:
        frames = scenes.fusion_frames(2, w, h, seed_offset=w * 1000 + h)
    else:  # too small for the depth-field generator: i.i.d. seeded primitives
        frames = [_tiny_frame(w, h, seed) for seed in (1, 2)]
    fu = Fusion(rast, w, h)
    for f in frames:
        for tau in (0.05, -1.0, 10.0):
            acc = torch.from_numpy(f.accum).cuda() if gate else None
            cnt = fu.run(_dev(f.planes), w, h, f.s, f.q, f.t, tau, acc, 0.5)
            torch.cuda.synchronize()
            ref = fusion.voxelize_fuse(w, h, f.planes, float(np.float32(f.s)), f.q.astype(np.float64),
                                       f.t.astype(np.float64), float(np.float32(tau)),
                                       f.accum if gate else None, float(np.float32(0.5)))
            n = ref["opacity"].size
            assert int(cnt.item()) == n, (w, h, tau, gate)
            if n:
                _check(fu, ref, n)


def test_fusion_capacity_and_errors(rast):
    w, h = 33, 21
    f = scenes.fusion_frames(1, w, h)[0]
    planes = _dev(f.planes)
    ref = fusion.voxelize_fuse(w, h, f.planes, float(np.float32(f.s)), f.q.astype(np.float64),
                               f.t.astype(np.float64), -1.0)
    cap = 100
    out = {k: torch.full((ref[k].reshape(-1, ref["opacity"].size).shape[0], cap + 8), -7.0, device="cuda")
           for k in PLANES}
    ws = torch.empty(int(rast.lib.fm_fusion_workspace_size(w, h)), dtype=torch.uint8, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    pm = native.FmPixelMap(w, h, *(planes[k].data_ptr() for k in PLANES))
    pose = native.FmSim3(f.s, (ctypes.c_float * 4)(*f.q), (ctypes.c_float * 3)(*f.t))
    fp = native.FmFusionParams(-1.0, 1.0)
    # planes of capacity `cap` laid out with stride cap (the extra columns must stay untouched)
    buf_t = {k: torch.full((out[k].shape[0] * cap + 64,), -7.0, device="cuda") for k in PLANES}
    buf = native.FmSurfelBuffer(*(buf_t[k].data_ptr() for k in PLANES), cap)
    rast.check(rast.lib.fm_voxelize_fuse(rast.ctx, ctypes.byref(pm), ctypes.byref(pose), ctypes.byref(fp), None,
                                         buf, _ptr(count), _ptr(ws), ws.numel(), None))
    torch.cuda.synchronize()
    assert int(count.item()) == w * h
    for k in PLANES:
        c = out[k].shape[0]
        got = buf_t[k][:c * cap].reshape(c, cap).cpu().numpy()
        np.testing.assert_allclose(got, ref[k].reshape(c, -1)[:, :cap], rtol=2e-6, atol=2e-5)
        assert torch.all(buf_t[k][c * cap:] == -7.0)
    bad_pose = native.FmSim3(0.0, (ctypes.c_float * 4)(1, 0, 0, 0), (ctypes.c_float * 3)(0, 0, 0))
    assert rast.lib.fm_voxelize_fuse(rast.ctx, ctypes.byref(pm), ctypes.byref(bad_pose), ctypes.byref(fp), None,
                                     buf, _ptr(count), _ptr(ws), ws.numel(), None) == native.FM_ERR_INVALID_ARG
    assert rast.lib.fm_voxelize_fuse(rast.ctx, ctypes.byref(pm), ctypes.byref(pose), ctypes.byref(fp), None,
                                     buf, _ptr(count), _ptr(ws), 0, None) == native.FM_ERR_WORKSPACE
    empty = native.FmPixelMap(0, h, *(planes[k].data_ptr() for k in PLANES))
    assert rast.lib.fm_voxelize_fuse(rast.ctx, ctypes.byref(empty), ctypes.byref(pose), ctypes.byref(fp), None,
                                     buf, _ptr(count), _ptr(ws), ws.numel(), None) == native.FM_ERR_INVALID_ARG


@pytest.mark.parametrize("tau", [0.05, -1.0])
def test_fusion_batch_equals_frames(rast, tau):
    """One fm_voxelize_fuse_batch over frames of mixed sizes (some gated,
    some not) writes exactly the concatenation of the per-frame calls, and
    its offsets delimit each frame's survivors."""
    shapes = [(64, 48), (65, 47), (9, 7), (1, 1), (33, 21), (2, 1)]
    frames = []
    for i, (w, h) in enumerate(shapes):
        if w >= 3 and h >= 3:
            frames.append(scenes.fusion_frames(1, w, h, seed_offset=500 + i)[0])
        else:
            frames.append(_tiny_frame(w, h, 40 + i))
    gates = [torch.from_numpy(f.accum).cuda() if i % 2 == 0 else None for i, f in enumerate(frames)]
    dev = [_dev(f.planes) for f in frames]
    print(f"fusion batch of {len(shapes)} frames tau={tau}", flush=True)
    fb = FusionBatch(rast, shapes)
    off = fb.run([(d, f.s, f.q, f.t) for d, f in zip(dev, frames)], tau, gates, 0.5)
    torch.cuda.synchronize()
    off = off.cpu().numpy()
    assert off[0] == 0 and np.all(np.diff(off) >= 0)
    for i, ((w, h), f, d, g) in enumerate(zip(shapes, frames, dev, gates)):
        fu = Fusion(rast, w, h)
        cnt = int(fu.run(d, w, h, f.s, f.q, f.t, tau, g, 0.5).item())
        torch.cuda.synchronize()
        assert off[i + 1] - off[i] == cnt, (i, off, cnt)
        for k in PLANES:
            a = fb.out[k][:, off[i]:off[i + 1]]
            b = fu.out[k].reshape(-1, fu.cap)[:, :cnt]
            assert torch.equal(a, b), (i, k)


def test_fusion_batch_errors(rast):
    w, h = 9, 7
    f = scenes.fusion_frames(1, w, h)[0]
    planes = _dev(f.planes)
    maps = (native.FmPixelMap * 2)(native.FmPixelMap(w, h, *(planes[k].data_ptr() for k in PLANES)),
                                   native.FmPixelMap(w, h, *(planes[k].data_ptr() for k in PLANES)))
    poses = (native.FmSim3 * 2)(native.FmSim3(f.s, (ctypes.c_float * 4)(*f.q), (ctypes.c_float * 3)(*f.t)),
                                native.FmSim3(f.s, (ctypes.c_float * 4)(*f.q), (ctypes.c_float * 3)(*f.t)))
    fp = native.FmFusionParams(0.05, 1.0)
    need = int(rast.lib.fm_fusion_batch_workspace_size(maps, 2))
    assert need > 0 and int(rast.lib.fm_fusion_batch_workspace_size(maps, 0)) == 0
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    cap = 2 * w * h
    out = {k: torch.empty(native_channels, cap, device="cuda") for k, native_channels in
           (("mean", 3), ("quat", 4), ("scale", 2), ("opacity", 1), ("color", 3))}
    buf = native.FmSurfelBuffer(*(out[k].data_ptr() for k in PLANES), cap)
    offs = torch.zeros(3, dtype=torch.int32, device="cuda")
    call = rast.lib.fm_voxelize_fuse_batch
    assert call(rast.ctx, maps, poses, 2, ctypes.byref(fp), None, buf, _ptr(offs), _ptr(ws), need, None) == 0
    torch.cuda.synchronize()
    o = offs.cpu().numpy()
    assert o[1] == o[2] - o[1] and o[2] <= cap  # the same frame twice
    assert call(rast.ctx, maps, poses, 0, ctypes.byref(fp), None, buf, _ptr(offs), _ptr(ws), need,
                None) == native.FM_ERR_INVALID_ARG
    assert call(rast.ctx, maps, poses, 2, ctypes.byref(fp), None, buf, None, _ptr(ws), need,
                None) == native.FM_ERR_INVALID_ARG
    assert call(rast.ctx, maps, poses, 2, ctypes.byref(fp), None, buf, _ptr(offs), _ptr(ws), need - 1,
                None) == native.FM_ERR_WORKSPACE
    poses[1] = native.FmSim3(-1.0, (ctypes.c_float * 4)(*f.q), (ctypes.c_float * 3)(*f.t))
    assert call(rast.ctx, maps, poses, 2, ctypes.byref(fp), None, buf, _ptr(offs), _ptr(ws), need,
                None) == native.FM_ERR_INVALID_ARG


def test_fusion_full_size_batch_matches_oracle(rast):
    """The benchmark's workload: one fm_voxelize_fuse_batch over 32 per-pixel
    maps of 518x392 with accumulation gates (tau_depth 0.05, gate 0.5);
    frames 0, 17 and 31 of the batch against the oracle (counts and order
    exact, values to float32 rounding), the offsets against the counts."""
    w, h, n_frames = 518, 392, 32
    print("fusion batch 32 x 518x392", flush=True)
    frames = scenes.fusion_frames(n_frames, w, h)
    dev = [_dev(f.planes) for f in frames]
    gates = [torch.from_numpy(f.accum).cuda() for f in frames]
    fb = FusionBatch(rast, [(w, h)] * n_frames)
    off = fb.run([(d, f.s, f.q, f.t) for d, f in zip(dev, frames)], 0.05, gates, 0.5)
    torch.cuda.synchronize()
    off = off.cpu().numpy()
    assert off[0] == 0 and np.all(np.diff(off) >= 0)
    for i in (0, 17, 31):
        f = frames[i]
        print(f"fusion oracle frame {i}", flush=True)
        ref = fusion.voxelize_fuse(w, h, f.planes, float(np.float32(f.s)), f.q.astype(np.float64),
                                   f.t.astype(np.float64), float(np.float32(0.05)), f.accum,
                                   float(np.float32(0.5)))
        n = ref["opacity"].size
        assert off[i + 1] - off[i] == n, (i, off[i + 1] - off[i], n)
        for k in PLANES:
            want = ref[k].reshape(-1, n)
            got = fb.out[k][:, off[i]:off[i + 1]].reshape(-1, n).cpu().numpy().astype(np.float64)
            tol = 2e-6 * (np.abs(want) + (1.0 if k == "mean" else 0.0) * 6.0) + 1e-7
            assert np.all(np.abs(got - want) <= tol), (i, k, np.max(np.abs(got - want) - tol))
