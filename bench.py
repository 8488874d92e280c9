#!/usr/bin/env python3
"""Benchmark of the MI355X 2DGS surfel rasterizer: forward + L1 render loss +
backward, in Mpixel/s and views/s, batched fused vs per-view plain.

Workload (default): 16 keyframes at 640x480 of the 300k-surfel scene
(config-1 laws: centres in [-3,3]^2 x [1,8], log-uniform tangent scales in
[0.01, 0.1], random rotations, sigmoid(N(0,1)) opacity, uniform colour),
poses along a smooth random trajectory, L1 RGB + 0.1 L1 depth against
seeded random targets.  One step = one pass of the whole hot path over the
batch: projection, depth sort, binning, tile sort, fused forward + loss +
backward blend, backward projection, gradients accumulated into the shared
surfel tensors and the 16 view matrices (zeroed at the start of each step).

  batched fused : one hipGraph replay of fm_fwd_bwd_l1 over all 16 views
  per-view plain: for each view fm_forward -> torch L1 gradient -> fm_backward

Prints one JSON line (rank 0) as the last line of stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "fwd+bwd Mpixel/s and views/s, batched fused vs per-view plain, 640x480"
# Algorithmic VALU lane-operations per useful (pixel, surfel) evaluation --
# inside the support and before termination: forward 32 + 2 transcendentals,
# backward 90 + 3 transcendentals, a transcendental counting 4 (quarter
# rate).  Tile over-evaluation and cross-lane reductions are not counted.
OPS_PER_USEFUL = 32 + 2 * 4 + 90 + 3 * 4
# gfx950: 256 CUs x 64 FP32 lanes x 2.4 GHz, one non-packed VALU op per lane per clock
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# The paper's own speed figures for the backend (appendix "Detailed Runtime
# Breakdown", runtime table; one RTX 4090 with a Xeon 6133, the experimental
# setup of Sec. 4).  Other hardware, and the keyframe count, resolution and
# map size of its refine step are not stated: context only, never a target.
PAPER_CONTEXT = dict(hardware="one RTX 4090 + Xeon 6133 (the paper's setup)",
                     refine_ms_per_frame=77.0, refine_iterations_per_frame=20,
                     refine_ms_per_iteration=77.0 / 20, merge_voxelization_ms_per_frame=0.5,
                     loop_correction_ms=2.0)
# HBM traffic of the blend kernel measured with rocprofv3 FETCH_SIZE / WRITE_SIZE
# (scaled by a 1 GiB copy), valid while the kernel source is the one measured
TRAFFIC_FILE = os.path.join(HERE, "profiles", "blend_traffic_headline.json")
BLEND_SOURCE = os.path.join(HERE, "paper_2604_03092_amd", "csrc", "fm_blend.hip")


def git_blob_sha1(path):
    """git's object id of a file (sha1 of 'blob <size>\\0' + bytes)."""
    import hashlib
    data = open(path, "rb").read()
    return hashlib.sha1(b"blob %d\0" % len(data) + data).hexdigest()


def blend_kernel_name(tw, th, waves, depth, deterministic):
    """The blend kernel's name as the profiler prints it for a launch."""
    split = "true" if waves == 2 else "false"
    det = "true" if deterministic else "false"
    return f"k_render_fused<Geo<{tw}, {th}, {split}, {depth}>, {det}>"


def measured_traffic(kernel, order):
    """Per-launch HBM bytes of the blend kernel, or None when the measurement
    is missing, was taken on a different kernel source, or on another launch
    (kernel instance or tile order) than the one timed."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("blend_source_sha1") != git_blob_sha1(BLEND_SOURCE):
        return None
    if t.get("kernel") != kernel or t.get("tile_order") != order:
        return None
    return t.get("bytes_per_launch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(name):
    from paper_2604_03092_amd import scenes
    return scenes.make(name)


def host_info():
    """CPU model, logical CPUs of the host, and CPUs this process may run on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    return dict(cpu_model=model, nproc=os.cpu_count(), cpus_allowed=allowed)


def _oracle_fwd_bwd(scene, n_views, threads):
    """Seconds of one FP64 oracle forward + L1 loss + backward of the first
    n_views views of the batch, and their pixel count."""
    import oracle
    from paper_2604_03092_amd import scenes as S
    npx = sum(w * h for (w, h, _) in scene.views[:n_views])
    sub = S.Scene("sample", scene.submaps, list(scene.views[:n_views]), scene.intr[:n_views],
                  scene.viewmat[:n_views], scene.target_rgb[:, :npx],
                  scene.target_depth[:npx] if scene.target_depth is not None else None, scene.w_rgb,
                  scene.w_depth)
    oracle.lib()
    t0 = time.perf_counter()
    out = oracle.render_scene(sub, n_threads=threads)
    _, g = oracle.l1_loss(sub, out)
    oracle.backward_scene(sub, g, n_threads=threads)
    return time.perf_counter() - t0, npx


def cpu_baseline(scene, threads, n_sample):
    """FP64 oracle (as it stands) on bounded samples of the batch: the first
    n_sample views on `threads` threads, and the first view on one thread."""
    n_sample = min(n_sample, scene.n_views)
    dt, npx = _oracle_fwd_bwd(scene, n_sample, threads)
    dt1, npx1 = _oracle_fwd_bwd(scene, 1, 1)
    w, h, s = scene.views[0]
    return dict(value=round(npx / dt / 1e6, 6), unit="Mpixel/s", cores=threads, kind="oracle",
                sample=f"views 0-{n_sample - 1} of {scene.n_views} ({w}x{h}, "
                       f"{scene.submaps[s]['opacity'].shape[0]} surfels): FP64 oracle forward + L1 loss + "
                       f"backward on {threads} threads, {dt:.2f} s",
                single_thread=dict(value=round(npx1 / dt1 / 1e6, 6), unit="Mpixel/s", cores=1,
                                   sample=f"view 0 on one thread, {dt1:.2f} s"),
                **host_info())


def time_refine(rast, scene, params, iters, replays=3):
    """The map-refinement loop over the batch's keyframes: `iters` iterations
    of (fused forward + L1 + backward storing the gradients, Adam step on
    every surfel tensor) captured in one hipGraph and replayed.  Every replay
    starts from the batch's initial surfels with fresh Adam state (restored
    outside the timed region), as a keyframe window's refinement does.  The
    pair buffer is sized from the largest pair count of an eager pass over
    all iterations (the map moves under Adam), checked after every one."""
    import torch
    from paper_2604_03092_amd.raster import Adam, GpuScene
    gs = GpuScene.from_scene(scene)
    init = [{k: sm[k].clone() for k in sm} for sm in gs.submaps]
    out, ws = rast.forward(gs, params)
    torch.cuda.synchronize()
    _, n_pairs, _ = rast.query(gs, ws)
    ws = rast.workspace(gs, params, max_pairs=int(n_pairs * 1.5) + 4096)
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    adam = Adam(rast, gs, grads)
    losses = torch.zeros(iters, device="cuda")

    def iteration(i):
        rast.fwd_bwd_l1(gs, ws, out, grads, dvm, losses[i:i + 1])
        adam.step()

    def restore():
        for sm, s0, m, v, g in zip(gs.submaps, init, adam.m, adam.v, grads):
            for k in sm:
                sm[k].copy_(s0[k])
                m[k].zero_()
                v[k].zero_()
                g[k].zero_()
        adam.step_count.zero_()
        losses.zero_()
        torch.cuda.synchronize()

    # eager pass: the largest pair count along the refinement trajectory
    max_req = 0
    for i in range(iters):
        iteration(i)
        torch.cuda.synchronize()
        st, _, req = rast.query(gs, ws)
        max_req = max(max_req, req)
    if max_req * 1.1 > ws.max_pairs:
        ws = rast.workspace(gs, params, max_pairs=int(max_req * 1.25) + 4096)
    restore()

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        iteration(0)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for i in range(iters):
            iteration(i)

    restore()
    graph.replay()  # warm-up replay
    torch.cuda.synchronize()
    first = float(losses[0])
    dt = 0.0
    for _ in range(replays):
        restore()
        t0 = time.perf_counter()
        graph.replay()
        torch.cuda.synchronize()
        dt += time.perf_counter() - t0
    dt /= replays * iters
    st, _, req = rast.query(gs, ws)
    return dict(iterations=iters, views=gs.n_views, ms_per_iteration=round(dt * 1e3, 4),
                ms_per_graph=round(dt * iters * 1e3, 3), mpixel_s=round(gs.npx / dt / 1e6, 3),
                loss_first=round(first, 6), loss_last=round(float(losses[-1]), 6),
                max_pairs_seen=int(max_req), pair_capacity=int(ws.max_pairs),
                pair_capacity_ok=bool(st == 0 and max_req <= ws.max_pairs))


def time_fusion(rast, n_frames=32, w=518, h=392, tau_depth=0.05, tau_accum=0.5, replays=20):
    """Map fusion of the incoming per-pixel maps of n_frames keyframes
    (2x2 adaptive voxelization, similarity to world, accumulation gate):
    all frames fused by one fm_voxelize_fuse_batch call, captured in a
    hipGraph and replayed."""
    import torch
    from paper_2604_03092_amd import scenes
    from paper_2604_03092_amd.raster import PLANES, FusionBatch
    frames = scenes.fusion_frames(n_frames, w, h)
    dev = [{k: torch.from_numpy(f.planes[k]).cuda() for k in PLANES} for f in frames]
    acc = [torch.from_numpy(f.accum).cuda() for f in frames]
    fb = FusionBatch(rast, [(w, h)] * n_frames)
    batch = [(d, f.s, f.q, f.t) for d, f in zip(dev, frames)]

    def run():
        fb.run(batch, tau_depth, acc, tau_accum)

    run()
    torch.cuda.synchronize()
    n_out = int(fb.offsets[-1].item())
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()
    torch.cuda.current_stream().wait_stream(s)
    with torch.cuda.graph(graph):
        run()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(replays):
        graph.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / replays
    npx = n_frames * w * h
    alg = 56 * npx + 52 * n_out   # 13 floats + accumulation in per pixel, 13 floats out per primitive
    return dict(frames=n_frames, size=f"{w}x{h}", pixels=npx, primitives_out=n_out, mode="one batched call",
                ms_per_batch=round(dt * 1e3, 4), mpixel_s=round(npx / dt / 1e6, 1),
                hbm=dict(bytes=alg, gbs=round(alg / dt / 1e9, 1), frac=round(alg / dt / 1e9 / HBM_PEAK_GBS, 4)))


def time_warp(rast, n=16_000_000, n_keyframes=64, replays=20):
    """Loop-correction warp (fm_warp_keyframes) of n keyframe-bound primitives
    by per-keyframe similarities: one launch, timed with events over replays.
    16M primitives are 1.2 GB of data, several times the 256 MB last-level
    cache, so every replay streams them from HBM."""
    import ctypes
    import numpy as np
    import torch
    from paper_2604_03092_amd import native
    from paper_2604_03092_amd.raster import _ptr
    rng = np.random.Generator(np.random.PCG64(30920 + 77))
    q = rng.normal(size=(4, n))
    mean = torch.from_numpy(rng.normal(0, 3, (3, n)).astype(np.float32)).cuda()
    quat = torch.from_numpy((q / np.linalg.norm(q, axis=0)).astype(np.float32)).cuda()
    scale = torch.from_numpy(rng.uniform(0.01, 0.1, (2, n)).astype(np.float32)).cuda()
    kf = torch.from_numpy(rng.integers(0, n_keyframes, n).astype(np.int32)).cuda()
    arr = (native.FmSim3 * n_keyframes)()
    for k in range(n_keyframes):
        # near-identity moves keep repeated replays bounded
        qq = np.array([1.0, *rng.normal(0, 1e-3, 3)])
        arr[k] = native.FmSim3(1.0, (ctypes.c_float * 4)(*qq), (ctypes.c_float * 3)(*rng.normal(0, 1e-3, 3)))
    deltas = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).cuda()

    def run():
        rast.check(rast.lib.fm_warp_keyframes(rast.ctx, _ptr(mean), _ptr(quat), _ptr(scale), _ptr(kf), n,
                                              _ptr(deltas), n_keyframes, None))

    run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(replays):
        run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / replays
    alg = n * (9 * 4 * 2 + 4)  # mean, quat, scale read and written, keyframe id read
    return dict(primitives=n, keyframes=n_keyframes, ms=round(ms, 4),
                hbm=dict(bytes=alg, gbs=round(alg / ms / 1e6, 1), frac=round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)))


def step_alg_bytes(n_surf, n_vis, n_pairs, npx):
    """Algorithmic HBM bytes of one fused step: 52 B of parameters read and
    52 B of gradients written per surfel; per visible (view, surfel) a 68 B
    record and a 68 B screen-space gradient, each written and read once; per
    pair 12 B emitted, 24 B for one sort pass, 4 B read by the forward and
    4 B by the backward traversal; per pixel 32 B of outputs, 8 B of state
    written and read, 32 B of upstream gradient (targets)."""
    return 104 * n_surf + 272 * n_vis + 44 * n_pairs + 80 * npx


def step_rooflines(n_surf, n_vis, n_pairs, npx, useful, ms):
    """The step's HBM fraction by the byte model and its VALU fraction by the
    useful evaluations, both over the whole step time."""
    b = step_alg_bytes(n_surf, n_vis, n_pairs, npx)
    t = ms * 1e-3
    ops = useful * OPS_PER_USEFUL
    return dict(hbm=dict(bytes=b, gbs=round(b / t / 1e9, 1), frac=round(b / t / 1e9 / HBM_PEAK_GBS, 4)),
                valu=dict(lane_ops=ops, tops=round(ops / t / 1e12, 3),
                          frac=round(ops / t / 1e12 / ALU_PEAK_TOPS, 4)))


def lds_peak(rast, blocks=256 * 8 * 4, iters=4096):
    """LDS read bandwidth measured with the library's probe (per-lane 16-byte
    words without bank conflicts, and wave broadcasts of one 16-byte word)."""
    import ctypes
    import torch
    sink = torch.empty(blocks * 256, device="cuda")
    res = {}
    for mode, name in ((0, "per_lane"), (1, "broadcast")):
        nbytes = ctypes.c_double(0)
        st = torch.cuda.current_stream()
        call = lambda: rast.check(rast.lib.fm_bench_lds(rast.ctx, mode, blocks, iters, ctypes.c_void_p(sink.data_ptr()),
                                                        ctypes.byref(nbytes), ctypes.c_void_p(st.cuda_stream)))
        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for _ in range(reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        insts = blocks * 4 * iters * 8   # wave-level ds_read_b128 instructions
        res[name] = dict(lane_tbs=round(nbytes.value / ms / 1e9, 2), ms=round(ms, 4),
                         wave_insts_per_s=float(f"{insts / ms * 1e3:.4g}"))
    res["nominal_tbs"] = round(256 * 128 * 2.4e9 / 1e12, 1)  # 128 B per clock per CU
    return res


def tune_launch(rast, gs, deterministic=False):
    """The autotuner's launch for a batch (untimed): (tile w, tile h, tile
    order, waves per tile, LDS depth).  Its workspace and pair capacity are
    sized for the largest candidate (8x8 tiles)."""
    import torch
    p8 = rast.params(tile=(8, 8), overwrite=True, deterministic=deterministic)
    _, ws8 = rast.forward(gs, p8)
    torch.cuda.synchronize()
    ws8 = rast.workspace(gs, p8, max_pairs=int(ws8.n_pairs * 1.1) + 4096)
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    loss = torch.zeros(1, device="cuda")
    c = rast.autotune(gs, ws8, out, grads, dvm, loss)
    del ws8, out, grads, dvm
    torch.cuda.empty_cache()
    return (int(c.tile_w), int(c.tile_h), int(c.tile_order), int(c.tile_waves), int(c.lds_depth))


def time_config(rast, name, steps):
    """Fused forward + L1 + backward of one config's whole batch, one hipGraph
    replay per step, at 16x16 tiles (longest list first) and at the tile shape
    and order the autotuner picks (setup, tuning and pair-buffer sizing
    untimed), each with the step's HBM and VALU rooflines."""
    import torch
    from paper_2604_03092_amd.raster import GpuScene
    scene = make_workload(name)
    gs = GpuScene.from_scene(scene)
    # the autotuner needs a workspace and capacity for its largest candidate (8x8)
    p8 = rast.params(tile=(8, 8), overwrite=True)
    _, ws8 = rast.forward(gs, p8)
    torch.cuda.synchronize()
    ws8 = rast.workspace(gs, p8, max_pairs=int(ws8.n_pairs * 1.1) + 4096)
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    loss = torch.zeros(1, device="cuda")
    chosen = rast.autotune(gs, ws8, out, grads, dvm, loss)
    tuned = (int(chosen.tile_w), int(chosen.tile_h), int(chosen.tile_order), int(chosen.tile_waves),
             int(chosen.lds_depth))
    del ws8
    res = dict(views=gs.n_views, pixels=gs.npx)
    default = (16, 16, 1, 1, 64)
    for launch in [default] + ([tuned] if tuned != default else []):
        r = _time_config_tile(rast, gs, launch, steps, out, grads, dvm, loss)
        key = "tile_16x16" if launch == default else "tuned"
        res[key] = dict(tile=f"{launch[0]}x{launch[1]}", **r)
    res["autotuned_tile"] = f"{tuned[0]}x{tuned[1]}"
    res["autotuned_order"] = "longest list first" if chosen.tile_order == 1 else "image order"
    res["autotuned_waves_per_tile"] = "one per 8x8 block" if chosen.tile_waves == 2 else "one per tile"
    res["autotuned_lds_depth"] = int(chosen.lds_depth)
    del out, grads, dvm
    torch.cuda.empty_cache()
    return res


def _time_config_tile(rast, gs, launch, steps, out, grads, dvm, loss):
    """One hipGraph replay of the fused step per timed step (gradients,
    pose gradients and loss stored), timed with events; the rooflines use the
    step's median time.  launch: (tile w, tile h, tile order, waves per
    tile, LDS batch depth)."""
    import torch
    tw, th, order, waves, depth = launch
    params = rast.params(tile=(tw, th), overwrite=True, tile_order=order, tile_waves=waves, lds_depth=depth)
    _, ws = rast.forward(gs, params)
    torch.cuda.synchronize()
    _, n_pairs, _ = rast.query(gs, ws)
    ws = rast.workspace(gs, params, max_pairs=int(n_pairs * 1.1) + 4096)

    def step():  # stores gradients, pose gradients and the loss (overwrite mode)
        rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss)

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    assert rast.query(gs, ws)[0] == 0
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    graph.replay()
    torch.cuda.synchronize()
    per, total = _timed_replays(graph.replay, steps)
    assert rast.query(gs, ws)[0] == 0
    med = float(np.median(per))
    # useful evaluations (contributor counts of a plain forward), visible entries
    rast.forward_into(gs, ws, out)
    torch.cuda.synchronize()
    _, nc = rast.pixel_state(gs, ws)
    useful = int(nc.astype(np.int64).sum())
    n_vis, _ = rast.counts(gs, ws)
    n_surf = sum(int(gs.submaps[k]["opacity"].shape[-1]) for k in {v[2] for v in gs.views})
    res = dict(pairs=n_pairs, visible_entries=n_vis, useful_evals=useful,
               ms_per_step=round(total / steps, 4), ms_per_step_median=round(med, 4),
               mpixel_s=round(gs.npx / med / 1e3, 3), views_s=round(gs.n_views / med * 1e3, 3),
               **step_rooflines(n_surf, n_vis, n_pairs, gs.npx, useful, med))
    del ws, graph
    torch.cuda.empty_cache()
    return res


def _timed_replays(run, steps):
    """Per-step milliseconds (events between consecutive runs on the current
    stream) and the total wall milliseconds of `steps` runs."""
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for i in range(steps):
        run()
        ev[i + 1].record()
    torch.cuda.synchronize()
    total = (time.perf_counter() - t0) * 1e3
    return [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)], total


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="headline")
    ap.add_argument("--tile", default="auto",
                    help="tile shape WxH, or auto: the autotuner picks the shape, tile order, waves per tile and "
                         "LDS depth for the batch (untimed) and the step runs with its choice")
    ap.add_argument("--tile-order", type=int, default=1, choices=(1, 2),
                    help="blend tile order: 1 longest list first, 2 image order")
    ap.add_argument("--tile-waves", type=int, default=1, choices=(1, 2),
                    help="blend waves per tile: 1 one per tile, 2 one per 8x8 block")
    ap.add_argument("--lds-depth", type=int, default=64, choices=(32, 64, 128),
                    help="records the fused blend stages in LDS per batch")
    ap.add_argument("--no-graph", action="store_true", help="time eager calls instead of a graph replay")
    ap.add_argument("--deterministic", action="store_true",
                    help="bitwise reproducible gradients (per-pair partials summed in a fixed order)")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-view plain comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--cpu-views", type=int, default=8, help="views in the CPU-baseline sample")
    ap.add_argument("--refine-iters", type=int, default=20,
                    help="iterations of the captured refine loop (render loss + Adam), 0 to skip")
    ap.add_argument("--no-fusion", action="store_true", help="skip the map-fusion and warp measurements")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the per-config block (configs 0-4, graph-replayed fused steps with rooflines)")
    ap.add_argument("--config-steps", type=int, default=20, help="timed steps per config and tile shape")
    ap.add_argument("--no-lds", action="store_true", help="skip the LDS bandwidth probe")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB device buffer 5 times (reference for HBM counter scaling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (views or submaps would shard "
              "across GPUs with one gradient all-reduce, see the design notes); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_03092_amd.raster import GpuScene, Rasterizer

    if args.copy_calibration:
        n = 1 << 28   # 2^28 float32 = 1 GiB
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": 4 * n, "copies": 5}), flush=True)
        return

    log(f"workload {args.workload}")
    scene = make_workload(args.workload)
    gs = GpuScene.from_scene(scene)
    rast = Rasterizer()
    # the step stores its gradients, pose gradients and loss (overwrite mode),
    # so no clearing kernels run between steps
    tuned = None
    if args.tile == "auto":
        from paper_2604_03092_amd import native
        try:
            tuned = tune_launch(rast, gs, args.deterministic)
        except native.FmError as e:  # e.g. no candidate fits the device memory: keep the default launch
            log(f"autotune failed ({e}); using 16x16, longest list first, one wave per tile, depth 64")
    if tuned is not None:
        tw, th, order, waves, depth = tuned
        log(f"autotuned: {tw}x{th}, order {order}, waves {waves}, lds depth {depth}")
    elif args.tile == "auto":
        tw, th, order, waves, depth = 16, 16, 1, 1, 64
    else:
        tw, th = (int(x) for x in args.tile.split("x"))
        order, waves, depth = args.tile_order, args.tile_waves, args.lds_depth
    params = rast.params(tile=(tw, th), deterministic=args.deterministic, overwrite=True, tile_order=order,
                         tile_waves=waves, lds_depth=depth)

    # size the pair buffer from one eager forward (not timed)
    out, ws = rast.forward(gs, params)
    torch.cuda.synchronize()
    _, n_pairs, _ = rast.query(gs, ws)
    ws = rast.workspace(gs, params, max_pairs=int(n_pairs * 1.1) + 4096)
    out = rast.new_outputs(gs)
    grads, dvm = gs.zero_grads()
    loss = torch.zeros(1, device="cuda")
    log(f"{gs.n_views} views, {gs.npx} px, {n_pairs} pairs, workspace {ws.nbytes / 2**20:.0f} MiB")

    def step():
        rast.fwd_bwd_l1(gs, ws, out, grads, dvm, loss)

    step()
    torch.cuda.synchronize()
    st, n_pairs, req = rast.query(gs, ws)
    assert st == 0, "pair capacity overflow"

    # per-phase timing of the eager fused path (HIP events between phases on
    # the call's stream); the blend kernel is the dominant one
    rast.set_timing(True)
    acc = None
    n_t = max(3, min(args.steps, 10))
    for _ in range(n_t):
        step()
        ph = rast.phase_times()
        acc = ph if acc is None else {k: acc[k] + ph[k] for k in acc}
    rast.set_timing(False)
    phases = {k: v / n_t for k, v in acc.items()}
    # contributor counts come from a plain forward (the fused path does not count)
    rast.forward_into(gs, ws, out)
    torch.cuda.synchronize()
    tf, nc = rast.pixel_state(gs, ws)
    useful = int(nc.astype(np.int64).sum())
    log(f"phases (ms): " + ", ".join(f"{k}={v:.3f}" for k, v in phases.items()))

    graph = None
    if not args.no_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(2):
                step()
        torch.cuda.current_stream().wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        torch.cuda.synchronize()

    run = graph.replay if graph is not None else step
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    log(f"timing {args.steps} fused steps ({'graph' if graph else 'eager'})")
    per_step, total_ms = _timed_replays(run, args.steps)
    dt = total_ms * 1e-3
    ms_step = dt / args.steps * 1e3
    ms_median = float(np.median(per_step))
    mpx = gs.npx * args.steps / dt / 1e6
    views_s = gs.n_views * args.steps / dt
    log(f"fused: {ms_step:.3f} ms/step, {mpx:.1f} Mpixel/s, {views_s:.1f} views/s")

    plain = None
    if not args.no_plain:
        plain_params = rast.params(tile=(16, 16), deterministic=args.deterministic)
        singles = []
        for v in range(gs.n_views):
            gv = GpuScene(gs.submaps, [gs.views[v]], gs.intr[v:v + 1].contiguous(), gs.viewmat[v:v + 1].contiguous())
            o = gs.pixel_offsets[v]
            npx = gv.npx
            tr = gs.target_rgb[:, o:o + npx].contiguous()
            td = gs.target_depth[o:o + npx].contiguous() if gs.target_depth is not None else None
            # per-view calls accumulate into the shared gradients
            o1, w1 = rast.forward(gv, plain_params)
            w1 = rast.workspace(gv, plain_params, max_pairs=int(w1.n_pairs * 1.1) + 4096)
            d1 = torch.zeros(1, 12, device="cuda")
            singles.append((gv, w1, rast.new_outputs(gv), tr, td, npx, d1))

        def plain_step():
            for g in grads:
                for t in g.values():
                    t.zero_()
            for (gv, w1, o1, tr, td, npx, d1) in singles:
                rast.forward_into(gv, w1, o1)
                k = gs.w_rgb / (3.0 * npx)
                g = dict(rgb=torch.sign(o1["rgb"] - tr) * k)
                if td is not None and gs.w_depth != 0.0:
                    g["depth"] = torch.sign(o1["depth"] - td) * (gs.w_depth / npx)
                d1.zero_()
                rast.backward(gv, w1, o1, g, grads, d1)

        for _ in range(max(1, args.warmup)):
            plain_step()
        torch.cuda.synchronize()
        for (gv, w1, *_rest) in singles:
            assert rast.query(gv, w1)[0] == 0
        k_plain = max(3, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(k_plain):
            plain_step()
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0
        plain = dict(ms_per_step=round(dtp / k_plain * 1e3, 4), mpixel_s=round(gs.npx * k_plain / dtp / 1e6, 3),
                     views_s=round(gs.n_views * k_plain / dtp, 3), steps=k_plain)
        log(f"plain: {plain['ms_per_step']:.3f} ms/step, {plain['mpixel_s']:.1f} Mpixel/s")

    blend_s = phases["blend"] * 1e-3
    blend_kernel = blend_kernel_name(tw, th, waves, 64 if args.deterministic else depth, args.deterministic)
    achieved = useful * OPS_PER_USEFUL / blend_s / 1e12 if blend_s > 0 else 0.0
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=round(ALU_PEAK_TOPS, 3), unit="TOP/s",
                    frac=round(achieved / ALU_PEAK_TOPS, 4), traffic=measured_traffic(blend_kernel, order),
                    kernel=blend_kernel, kernel_ms=round(phases["blend"], 4),
                    useful_evals=useful, ops_per_useful=OPS_PER_USEFUL)

    # HBM-bound phases against their algorithmic bytes: projection 52 B of
    # parameters per surfel + a 68 B record per visible (view, surfel);
    # binning 12 B emitted + 24 B of one sort pass per pair; backward
    # projection a 68 B screen-space gradient per visible entry + 52 B of
    # parameters read and 52 B of gradients written per surfel
    n_vis, _ = rast.counts(gs, ws)
    n_surf = int(sum(sm["opacity"].shape[0] for sm in scene.submaps))
    step_roof = step_rooflines(n_surf, n_vis, n_pairs, gs.npx, useful, ms_median)
    alg = {"projection": 52 * n_surf + 68 * n_vis, "binning": 36 * n_pairs,
           "backward_projection": 68 * n_vis + 104 * n_surf}
    phase_hbm = {k: dict(bytes=b, gbs=round(b / (phases[k] * 1e-3) / 1e9, 1),
                         frac=round(b / (phases[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
                 for k, b in alg.items() if phases.get(k, 0) > 0}

    refine = None
    if args.refine_iters > 0:
        refine = time_refine(rast, scene, params, args.refine_iters)
        log(f"refine: {refine['ms_per_iteration']:.3f} ms/iteration, {refine['mpixel_s']:.1f} Mpixel/s")

    fusion = None
    if not args.no_fusion:
        fusion = time_fusion(rast)
        log(f"fusion: {fusion['ms_per_batch']:.3f} ms for {fusion['frames']} frames, {fusion['mpixel_s']:.0f} Mpixel/s")

    warp = None
    if not args.no_fusion:
        warp = time_warp(rast)
        log(f"warp: {warp['ms']:.3f} ms for {warp['primitives']} primitives, {warp['hbm']['gbs']:.0f} GB/s")

    per_config = None
    if not args.no_configs:
        per_config = {}
        from paper_2604_03092_amd import native
        for name in ("config0", "config1", "config2", "config3", "config4"):
            log(f"config {name}")
            try:
                per_config[name] = time_config(rast, name, args.config_steps)
            except native.FmError as e:  # reported in the line; the headline measurement stands
                log(f"config {name} failed: {e}")
                per_config[name] = dict(error=str(e))

    lds = None
    if not args.no_lds:
        lds = lds_peak(rast)
        log(f"lds: per-lane {lds['per_lane']['lane_tbs']} TB/s, broadcast {lds['broadcast']['lane_tbs']} TB/s")

    cpu = None
    if not args.no_cpu_baseline:
        # every CPU this process may run on (the OpenMP thread budget when one is set)
        threads = args.cpu_threads or int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or host_info()["cpus_allowed"]
        log(f"cpu baseline on {threads} threads")
        cpu = cpu_baseline(scene, threads, args.cpu_views)

    res = {
        "metric": METRIC,
        "value": round(mpx, 3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "ms_per_step_median": round(ms_median, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": scene.name, "views": gs.n_views, "pixels_per_step": gs.npx,
                   "surfels": int(sum(sm["opacity"].shape[0] for sm in scene.submaps)),
                   "tile": f"{tw}x{th}", "mode": "hipgraph" if graph is not None else "eager",
                   "deterministic": bool(args.deterministic),
                   "tile_order": "longest list first" if order == 1 else "image order",
                   "waves_per_tile": "one per 8x8 block" if waves == 2 else "one per tile",
                   "lds_depth": depth,
                   "launch": "autotuned" if tuned else ("default (autotune failed)" if args.tile == "auto" else "given"),
                   "pairs": n_pairs},
        "views_per_s": round(views_s, 3),
        "plain": plain,
        "speedup_vs_plain": round(plain["ms_per_step"] / ms_step, 3) if plain else None,
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "visible_entries": n_vis,
        "phase_hbm": phase_hbm,
        "step_roofline": step_roof,
        "roofline": roofline,
        "lds": lds,
        "cpu_baseline": cpu,
        "refine": refine,
        "fusion": fusion,
        "warp": warp,
        "paper_context": dict(PAPER_CONTEXT,
                              this_refine_ms_per_iteration=refine["ms_per_iteration"] if refine else None,
                              this_fusion_ms_per_frame=(round(fusion["ms_per_batch"] / fusion["frames"], 5)
                                                        if fusion else None),
                              this_warp_ms=warp["ms"] if warp else None),
    }
    if per_config is not None:
        res["per_config"] = per_config
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
