"""GPU parity of the loop-correction warp (fm_warp_keyframes through the C
ABI) against the FP64 warp oracle."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import warp
from paper_2604_03092_amd import native
from paper_2604_03092_amd.raster import Rasterizer, _ptr, sim3_table, warp_keyframes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rast():
    return Rasterizer()


@pytest.mark.parametrize("n,K", [(0, 3), (1, 1), (100_003, 5), (65_537, 300)])
def test_warp_matches_oracle(rast, n, K):
    print(f"warp n={n} K={K}", flush=True)
    rng = np.random.default_rng(n + K)
    q = rng.normal(size=(4, n))
    planes = dict(mean=rng.normal(0, 3, (3, n)).astype(np.float32),
                  quat=(q / np.maximum(np.linalg.norm(q, axis=0), 1e-12)).astype(np.float32),
                  scale=rng.uniform(0.01, 0.1, (2, n)).astype(np.float32))
    kf = rng.integers(-1, K + 1, n).astype(np.int32)
    deltas = []
    arr = (native.FmSim3 * K)()
    for k in range(K):
        qq = rng.normal(size=4)
        s, t = float(rng.uniform(0.8, 1.2)), rng.normal(0, 1, 3)
        arr[k] = native.FmSim3(s, (ctypes.c_float * 4)(*qq), (ctypes.c_float * 3)(*t))
        deltas.append((float(np.float32(s)), qq.astype(np.float32).astype(np.float64),
                       t.astype(np.float32).astype(np.float64)))
    dev = {k: torch.from_numpy(v.copy()).cuda() if n else torch.zeros(1, device="cuda") for k, v in planes.items()}
    kf_d = torch.from_numpy(kf).cuda() if n else torch.zeros(1, dtype=torch.int32, device="cuda")
    d_d = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).cuda()
    rast.check(rast.lib.fm_warp_keyframes(rast.ctx, _ptr(dev["mean"]), _ptr(dev["quat"]), _ptr(dev["scale"]),
                                          _ptr(kf_d), n, _ptr(d_d), K, None))
    torch.cuda.synchronize()
    if n == 0:
        return
    ref = warp.warp(planes, kf, deltas)
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in dev.items()}
    np.testing.assert_allclose(got["mean"], ref["mean"], rtol=2e-6, atol=2e-5)
    np.testing.assert_allclose(got["quat"], ref["quat"], rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose(got["scale"], ref["scale"], rtol=2e-6)
    unbound = (kf < 0) | (kf >= K)
    for k in planes:
        np.testing.assert_array_equal(got[k][:, unbound], planes[k][:, unbound].astype(np.float64))


def test_warp_invalid_arguments(rast):
    x = torch.zeros(8, device="cuda")
    assert rast.lib.fm_warp_keyframes(rast.ctx, _ptr(x), None, _ptr(x), _ptr(x), 2, _ptr(x), 1, None) == \
        native.FM_ERR_INVALID_ARG
    assert rast.lib.fm_warp_keyframes(rast.ctx, _ptr(x), _ptr(x), _ptr(x), _ptr(x), 2, None, 1, None) == \
        native.FM_ERR_INVALID_ARG
    assert rast.lib.fm_warp_keyframes(rast.ctx, _ptr(x), _ptr(x), _ptr(x), _ptr(x), -1, _ptr(x), 1, None) == \
        native.FM_ERR_INVALID_ARG


def test_warp_wrapper_matches_oracle(rast):
    """The Python wrapper (sim3_table + warp_keyframes) on a small set."""
    rng = np.random.default_rng(91)
    n, K = 5000, 7
    q = rng.normal(size=(4, n))
    planes = dict(mean=rng.normal(0, 3, (3, n)).astype(np.float32),
                  quat=(q / np.linalg.norm(q, axis=0)).astype(np.float32),
                  scale=rng.uniform(0.01, 0.1, (2, n)).astype(np.float32))
    kf = rng.integers(-2, K + 2, n).astype(np.int32)
    host = [(float(rng.uniform(0.8, 1.2)), rng.normal(size=4), rng.normal(0, 1, 3)) for _ in range(K)]
    dev = {k: torch.from_numpy(v.copy()).cuda() for k, v in planes.items()}
    warp_keyframes(rast, dev, torch.from_numpy(kf).cuda(), sim3_table(host))
    torch.cuda.synchronize()
    deltas = [(float(np.float32(s)), np.asarray(qq, np.float32).astype(np.float64),
               np.asarray(t, np.float32).astype(np.float64)) for (s, qq, t) in host]
    ref = warp.warp(planes, kf, deltas)
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in dev.items()}
    np.testing.assert_allclose(got["mean"], ref["mean"], rtol=2e-6, atol=2e-5)
    np.testing.assert_allclose(got["quat"], ref["quat"], rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose(got["scale"], ref["scale"], rtol=2e-6)


def test_warp_full_size_sampled(rast):
    """The benchmark's size: 16M primitives bound to 64 keyframes (and a
    share unbound), warped in one launch; 200k sampled primitives against the
    oracle, computed on the sample alone (the warp is elementwise)."""
    n, K = 16_000_000, 64
    print(f"warp n={n} K={K}", flush=True)
    rng = np.random.default_rng(16064)
    q = rng.normal(size=(4, n)).astype(np.float32)
    q /= np.maximum(np.linalg.norm(q, axis=0), 1e-12)
    planes = dict(mean=rng.normal(0, 3, (3, n)).astype(np.float32), quat=q,
                  scale=rng.uniform(0.01, 0.1, (2, n)).astype(np.float32))
    kf = rng.integers(-1, K + 1, n).astype(np.int32)
    arr = (native.FmSim3 * K)()
    deltas = []
    for k in range(K):
        qq = rng.normal(size=4)
        s, t = float(rng.uniform(0.8, 1.2)), rng.normal(0, 1, 3)
        arr[k] = native.FmSim3(s, (ctypes.c_float * 4)(*qq), (ctypes.c_float * 3)(*t))
        deltas.append((float(np.float32(s)), qq.astype(np.float32).astype(np.float64),
                       t.astype(np.float32).astype(np.float64)))
    dev = {k: torch.from_numpy(v).cuda() for k, v in planes.items()}
    kf_d = torch.from_numpy(kf).cuda()
    d_d = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).cuda()
    rast.check(rast.lib.fm_warp_keyframes(rast.ctx, _ptr(dev["mean"]), _ptr(dev["quat"]), _ptr(dev["scale"]),
                                          _ptr(kf_d), n, _ptr(d_d), K, None))
    torch.cuda.synchronize()
    idx = np.sort(rng.choice(n, 200_000, replace=False))
    sub = {k: np.ascontiguousarray(v[:, idx]) for k, v in planes.items()}
    ref = warp.warp(sub, kf[idx], deltas)
    idx_d = torch.from_numpy(idx).cuda()
    got = {k: v[:, idx_d].cpu().numpy().astype(np.float64) for k, v in dev.items()}
    np.testing.assert_allclose(got["mean"], ref["mean"], rtol=2e-6, atol=2e-5)
    np.testing.assert_allclose(got["quat"], ref["quat"], rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose(got["scale"], ref["scale"], rtol=2e-6)
    unbound = (kf[idx] < 0) | (kf[idx] >= K)
    for k in planes:
        np.testing.assert_array_equal(got[k][:, unbound], sub[k][:, unbound].astype(np.float64))
