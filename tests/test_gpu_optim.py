"""GPU parity of the fused Adam step (fm_adam_step through the C ABI)
against the FP64 optimizer oracle, and the refine loop (render loss +
optimizer step) replayed from one captured graph."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import optim
from paper_2604_03092_amd import native, scenes
from paper_2604_03092_amd.raster import ADAM_KINDS, Adam, GpuScene, Rasterizer, _ptr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rast():
    return Rasterizer()


def _say(msg):
    print(msg, flush=True)


def _descriptor(p, g, m, v, lr, kind):
    return native.FmAdamTensor(p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), p.numel(), lr, kind)


@pytest.mark.parametrize("kind", [optim.LINEAR, optim.LOG, optim.LOGIT])
def test_adam_matches_oracle(rast, kind):
    """Three consecutive calls (device step counter 1, 2, 3) on tensors of
    ragged sizes; each call is compared with the oracle's step from the
    GPU's state before the call, so every comparison sees one step's
    rounding."""
    rng = np.random.default_rng(100 + kind)
    sizes = [0, 1, 257, 65539]
    lrs = [0.01, 0.02, 0.005, 0.03]
    dev = []
    for n in sizes:
        p = (rng.uniform(0.02, 0.98, n) if kind != optim.LINEAR else rng.normal(0, 1, n)).astype(np.float32)
        z = lambda: torch.zeros(max(n, 1), device="cuda")
        d = [z(), z(), z(), z()]
        d[0][:n] = torch.from_numpy(p).cuda()
        dev.append(d)
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    cfg = native.FmAdamConfig(0.9, 0.999, 1e-8)
    f32 = lambda x: float(np.float32(x))  # the oracle sees the float32 values the API carries
    for t in range(1, 4):
        _say(f"adam kind={kind} step {t}")
        arr = (native.FmAdamTensor * len(sizes))()
        expect = []
        for i, n in enumerate(sizes):
            g = (rng.normal(0, 1, n) * 10.0 ** rng.uniform(-3, 1, n)).astype(np.float32)
            dev[i][1][:n] = torch.from_numpy(g).cuda()
            p0, m0, v0 = (dev[i][k][:n].cpu().numpy().astype(np.float64) for k in (0, 2, 3))
            p1, m1, v1 = optim.adam_step(p0, g.astype(np.float64), m0, v0, t, f32(lrs[i]), kind, beta1=f32(0.9),
                                         beta2=f32(0.999), eps=f32(1e-8))
            _, gt = optim.to_theta(p0, g, kind)
            # FP32 rounding bounds: a few ulps of the terms each moment sums;
            # the step lr * m_hat / (sqrt(v_hat) + eps) is O(lr)
            expect.append((p1, m1, v1, 0.9 * np.abs(m0) + 0.1 * np.abs(gt), 0.999 * v0 + 0.001 * gt * gt))
            d = dev[i]
            arr[i] = native.FmAdamTensor(d[0].data_ptr(), d[1].data_ptr(), d[2].data_ptr(), d[3].data_ptr(),
                                         n, lrs[i], kind)
        rast.check(rast.lib.fm_adam_step(rast.ctx, arr, len(sizes), ctypes.byref(cfg), _ptr(step), None))
        torch.cuda.synchronize()
        for i, n in enumerate(sizes):
            p1, m1, v1, sm, sv = expect[i]
            gp, gm, gv = (dev[i][k][:n].cpu().numpy() for k in (0, 2, 3))
            assert np.all(np.abs(gm - m1) <= 1e-6 * sm + 1e-30), (kind, n, t)
            assert np.all(np.abs(gv - v1) <= 1e-6 * sv + 1e-30), (kind, n, t)
            assert np.all(np.abs(gp - p1) <= 2e-6 * np.abs(p1) + 1e-5 * lrs[i]), (kind, n, t)
    assert int(step.item()) == 3


def test_adam_many_tensors_and_zero_grad(rast):
    """20 tensors in one call (more than one launch's table) with gradient
    clearing: parameters and moments are bit-identical to the same step
    without clearing, and every gradient is zero afterwards."""
    rng = np.random.default_rng(7)
    sizes = [int(x) for x in rng.integers(0, 3000, 20)]
    kinds = [int(x) for x in rng.integers(0, 3, 20)]
    runs = []
    for zero in (0, 1):
        dev = []
        arr = (native.FmAdamTensor * len(sizes))()
        r2 = np.random.default_rng(8)
        for i, (n, k) in enumerate(zip(sizes, kinds)):
            p = (r2.uniform(0.02, 0.98, n) if k != optim.LINEAR else r2.normal(0, 1, n)).astype(np.float32)
            g = r2.normal(0, 1, n).astype(np.float32)
            d = [torch.from_numpy(p).cuda() if n else torch.zeros(1, device="cuda"),
                 torch.from_numpy(g).cuda() if n else torch.zeros(1, device="cuda"),
                 torch.zeros(max(n, 1), device="cuda"), torch.zeros(max(n, 1), device="cuda")]
            dev.append(d)
            arr[i] = native.FmAdamTensor(*(t.data_ptr() for t in d), n, 0.01, k)
        step = torch.zeros(1, dtype=torch.int32, device="cuda")
        cfg = native.FmAdamConfig(0.9, 0.999, 1e-8, zero)
        rast.check(rast.lib.fm_adam_step(rast.ctx, arr, len(sizes), ctypes.byref(cfg), _ptr(step), None))
        torch.cuda.synchronize()
        runs.append(dev)
    for i, n in enumerate(sizes):
        if n == 0:
            continue
        for j in (0, 2, 3):
            assert torch.equal(runs[0][i][j][:n], runs[1][i][j][:n]), (i, j)
        assert torch.count_nonzero(runs[1][i][1][:n]) == 0
        assert torch.count_nonzero(runs[0][i][1][:n]) > 0


def test_adam_invalid_arguments(rast):
    p = torch.zeros(4, device="cuda")
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    cfg = native.FmAdamConfig(0.9, 0.999, 1e-8)
    good = _descriptor(p, p, p, p, 0.1, optim.LINEAR)
    bad = [native.FmAdamTensor(p.data_ptr(), None, p.data_ptr(), p.data_ptr(), 4, 0.1, 0),
           _descriptor(p, p, p, p, 0.0, optim.LINEAR), _descriptor(p, p, p, p, 0.1, 7)]
    for d in bad:
        arr = (native.FmAdamTensor * 2)(good, d)
        assert rast.lib.fm_adam_step(rast.ctx, arr, 2, ctypes.byref(cfg), _ptr(step), None) == \
            native.FM_ERR_INVALID_ARG
    arr = (native.FmAdamTensor * 1)(good)
    for c in (native.FmAdamConfig(1.0, 0.999, 1e-8), native.FmAdamConfig(0.9, 0.999, 0.0)):
        assert rast.lib.fm_adam_step(rast.ctx, arr, 1, ctypes.byref(c), _ptr(step), None) == \
            native.FM_ERR_INVALID_ARG
    assert rast.lib.fm_adam_step(rast.ctx, arr, 1, ctypes.byref(cfg), None, None) == native.FM_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert int(step.item()) == 0  # nothing was launched


def test_refine_loop_in_one_graph(rast):
    """Render loss + Adam over the batch, iterated inside one captured graph:
    the loss falls, the step counter advances once per iteration and the
    parameters stay in their domains."""
    sc = scenes.config0()
    gs = GpuScene.from_scene(sc)
    params = rast.params()
    out, ws = rast.forward(gs, params)
    torch.cuda.synchronize()
    _, n_pairs, _ = rast.query(gs, ws)
    ws = rast.workspace(gs, params, max_pairs=2 * n_pairs + 4096)
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    adam = Adam(rast, gs, grads, lr=dict(color=0.02, opacity=0.05))
    iters = 10
    losses = torch.zeros(iters, device="cuda")

    def iteration(i):
        for g in grads:
            for t in g.values():
                t.zero_()
        dvm.zero_()
        rast.fwd_bwd_l1(gs, ws, out, grads, dvm, losses[i:i + 1])
        adam.step()

    _say("refine: warm-up and capture")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        iteration(0)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    losses.zero_()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for i in range(iters):
            iteration(i)
    torch.cuda.synchronize()
    _say("refine: replay")
    for rep in range(2):
        losses.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert rast.query(gs, ws)[0] == 0
        lh = losses.cpu().numpy()
        assert np.all(np.isfinite(lh)) and lh[-1] < lh[0], lh
    assert int(adam.step_count.item()) == 1 + 2 * iters
    for sm in gs.submaps:
        assert torch.isfinite(sm["mean"]).all() and torch.isfinite(sm["color"]).all()
        assert (sm["opacity"] > 0).all() and (sm["opacity"] < 1).all() and (sm["scale"] > 0).all()


def test_adam_full_size_chain(rast):
    """The refine loop's optimizer at full size: Adam over every tensor of
    the 300k-surfel scene (3.9M parameters in five tensors, the three
    parameter kinds) through the same binding the refine loop uses, three
    consecutive steps with seeded gradients (a third of the surfels get
    none, as unseen surfels do), each compared element by element with the
    oracle's chain of three steps from the same initial state.  The bounds
    grow with the step number: every step adds one step's FP32 rounding."""
    sc = scenes.config1()
    gs = GpuScene.from_scene(sc)
    grads, _ = gs.zero_grads()
    adam = Adam(rast, gs, grads)
    rng = np.random.default_rng(2024)
    f32 = lambda x: float(np.float32(x))
    state = {k: (sc.submaps[0][k].astype(np.float64), 0.0, 0.0, 0.0, 0.0) for k in gs.submaps[0]}
    n = gs.submaps[0]["opacity"].numel()
    for t in range(1, 4):
        _say(f"adam full size step {t}")
        seen = rng.random(n) < 2.0 / 3.0
        gnp = {}
        for k, gt in grads[0].items():
            g = rng.normal(0, 1, gt.shape) * 10.0 ** rng.uniform(-6, -1, gt.shape)
            g = (g * seen).astype(np.float32)
            gt.copy_(torch.from_numpy(g))
            gnp[k] = g
        adam.step()
        torch.cuda.synchronize()
        for k, (p0, m0, v0, sm0, sv0) in state.items():
            kind = int(ADAM_KINDS[k])
            p1, m1, v1 = optim.adam_step(p0, gnp[k].astype(np.float64), m0, v0, t, f32(adam.lr[k]), kind,
                                         beta1=f32(0.9), beta2=f32(0.999), eps=f32(1e-8))
            _, gth = optim.to_theta(p0, gnp[k], kind)
            sm1 = 0.9 * sm0 + 0.1 * np.abs(gth)
            sv1 = 0.999 * sv0 + 0.001 * gth * gth
            gp, gm, gv = (x[0][k].cpu().numpy() for x in (gs.submaps, adam.m, adam.v))
            dp = np.abs(gp - p1) - t * (2e-6 * np.abs(p1) + 1e-5 * adam.lr[k])
            assert dp.max() <= 0, (k, t, float(dp.max()))
            assert np.all(np.abs(gm - m1) <= 4e-6 * t * sm1 + 1e-30), (k, t)
            assert np.all(np.abs(gv - v1) <= 4e-6 * t * sv1 + 1e-30), (k, t)
            state[k] = (p1, m1, v1, sm1, sv1)
    assert int(adam.step_count.item()) == 3


def test_adam_unaligned_views_match_aligned(rast):
    """Buffers that are not 16-byte aligned take the element-by-element path;
    each of the three kinds gives the same parameters and moments as the
    same step on aligned buffers (which take the four-wide path)."""
    rng = np.random.default_rng(31)
    n = 5000
    step_a = torch.zeros(1, dtype=torch.int32, device="cuda")
    step_u = torch.zeros(1, dtype=torch.int32, device="cuda")
    cfg = native.FmAdamConfig(0.9, 0.999, 1e-8)
    for kind in (optim.LINEAR, optim.LOG, optim.LOGIT):
        p = (rng.uniform(0.02, 0.98, n) if kind != optim.LINEAR else rng.normal(0, 1, n)).astype(np.float32)
        g = rng.normal(0, 1, n).astype(np.float32)
        m = rng.normal(0, 0.1, n).astype(np.float32)
        v = rng.uniform(0, 0.1, n).astype(np.float32)
        al = [torch.from_numpy(x.copy()).cuda() for x in (p, g, m, v)]
        un = []
        for x in (p, g, m, v):
            buf = torch.zeros(n + 1, device="cuda")
            buf[1:] = torch.from_numpy(x)
            un.append(buf[1:])
        assert all(t.data_ptr() % 16 != 0 for t in un) and all(t.data_ptr() % 16 == 0 for t in al)
        for ts, st in ((al, step_a), (un, step_u)):
            arr = (native.FmAdamTensor * 1)(_descriptor(*ts, 0.01, kind))
            rast.check(rast.lib.fm_adam_step(rast.ctx, arr, 1, ctypes.byref(cfg), _ptr(st), None))
        torch.cuda.synchronize()
        for a, u in zip(al, un):
            assert torch.equal(a, u), kind
