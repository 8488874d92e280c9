"""Seeded synthetic scenes for the surfel rasterizer.

This module only draws inputs: surfel maps, cameras, trajectories and loss
targets.  It holds none of the rasterizer's arithmetic, so both the FP64 CPU
oracle and the HIP path can be fed from it without sharing any of the method.

Every generator uses NumPy's PCG64 with a fixed seed (``30920 + config``,
targets ``seed + 1000``).  The workloads stand in for the paper's datasets
(ScanNet, BundleFusion, KITTI, TUM; Sec. 4.1), which are not reproduced here.

Conventions (shared by every consumer):

* surfel planes are SoA float32: ``mean[3,n]``, ``quat[4,n]`` (w,x,y,z, any
  non-zero norm), ``scale[2,n]`` (linear, > 0), ``opacity[n]`` (activated,
  in (0,1]), ``color[3,n]`` (RGB, degree 0);
* a view is ``(W, H, submap)``; ``intr[v] = (fx, fy, cx, cy)``;
  ``viewmat[v]`` is the world->camera ``[R|t]`` as 12 row-major floats;
* per-pixel planes of all views are concatenated view after view
  (``pixel_offset[v] = sum of W*H of earlier views``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 30920


@dataclass
class Scene:
    name: str
    submaps: list            # list of dict(mean, quat, scale, opacity, color)
    views: list              # list of (W, H, submap)
    intr: np.ndarray         # [V,4] float32
    viewmat: np.ndarray      # [V,12] float32
    target_rgb: np.ndarray = None    # [3, sum px] float32
    target_depth: np.ndarray = None  # [sum px] float32
    w_rgb: float = 1.0
    w_depth: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def n_views(self):
        return len(self.views)

    @property
    def pixel_offsets(self):
        off, out = 0, []
        for (w, h, _) in self.views:
            out.append(off)
            off += w * h
        return out

    @property
    def total_pixels(self):
        return sum(w * h for (w, h, _) in self.views)

    def view_pixels(self, v):
        w, h, _ = self.views[v]
        return w * h


# --------------------------------------------------------------------------
# elementary draws
# --------------------------------------------------------------------------

def _surfels(rng, n, lo, hi, scale_lo=0.01, scale_hi=0.1):
    """Random surfels with the laws of the small scenes: uniform centres in a
    box, log-uniform tangent scales, uniformly random rotations (normalised
    Gaussian 4-vectors), sigmoid(N(0,1)) opacity, uniform RGB."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    mean = (lo[:, None] + (hi - lo)[:, None] * rng.random((3, n))).astype(np.float32)
    scale = np.exp(rng.uniform(math.log(scale_lo), math.log(scale_hi), (2, n))).astype(np.float32)
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    quat = q.astype(np.float32)
    opacity = (1.0 / (1.0 + np.exp(-rng.standard_normal(n)))).astype(np.float32)
    color = rng.random((3, n)).astype(np.float32)
    return dict(mean=np.ascontiguousarray(mean), quat=np.ascontiguousarray(quat),
                scale=np.ascontiguousarray(scale), opacity=np.ascontiguousarray(opacity),
                color=np.ascontiguousarray(color))


def _rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def _rot_axis(axis, ang):
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    k = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + math.sin(ang) * k + (1 - math.cos(ang)) * (k @ k)


def _viewmat_from_cam(r_wc, c):
    """World->camera [R|t] from a camera->world rotation and camera centre."""
    r = r_wc.T
    t = -r @ c
    return np.concatenate([r, t[:, None]], axis=1).reshape(12)


def trajectory(rng, n):
    """Smooth random camera path: yaw swings +-30 deg as a sinusoid with a
    random phase; the position follows a damped random walk
    v_k = 0.7 v_{k-1} + 0.3 U(-0.5,0.5)^3, clamped to [-1.5,1.5]^2 x [-1,0.5].
    Returns [n,12] world->camera matrices."""
    phi = rng.uniform(0.0, 2.0 * math.pi)
    pos = np.zeros(3)
    vel = np.zeros(3)
    lo = np.array([-1.5, -1.5, -1.0])
    hi = np.array([1.5, 1.5, 0.5])
    out = []
    for k in range(n):
        yaw = math.radians(30.0) * math.sin(2.0 * math.pi * k / max(n, 1) + phi)
        vel = 0.7 * vel + 0.3 * rng.uniform(-0.5, 0.5, 3)
        pos = np.clip(pos + vel, lo, hi)
        out.append(_viewmat_from_cam(_rot_y(yaw), pos))
    return np.asarray(out, np.float64)


def quat_from_matrix(m):
    """Unit quaternions (w,x,y,z) from rotation matrices [..., 3, 3]."""
    m = np.asarray(m, np.float64)
    tr = m[..., 0, 0] + m[..., 1, 1] + m[..., 2, 2]
    q = np.empty(m.shape[:-2] + (4,))
    c0 = tr > 0
    c1 = (~c0) & (m[..., 0, 0] >= m[..., 1, 1]) & (m[..., 0, 0] >= m[..., 2, 2])
    c2 = (~c0) & (~c1) & (m[..., 1, 1] >= m[..., 2, 2])
    c3 = ~(c0 | c1 | c2)
    s = np.sqrt(np.maximum(tr[c0] + 1.0, 1e-300)) * 2
    q[c0] = np.stack([0.25 * s, (m[c0][:, 2, 1] - m[c0][:, 1, 2]) / s,
                      (m[c0][:, 0, 2] - m[c0][:, 2, 0]) / s, (m[c0][:, 1, 0] - m[c0][:, 0, 1]) / s], -1)
    mm = m[c1]
    s = np.sqrt(np.maximum(1.0 + mm[:, 0, 0] - mm[:, 1, 1] - mm[:, 2, 2], 1e-300)) * 2
    q[c1] = np.stack([(mm[:, 2, 1] - mm[:, 1, 2]) / s, 0.25 * s,
                      (mm[:, 0, 1] + mm[:, 1, 0]) / s, (mm[:, 0, 2] + mm[:, 2, 0]) / s], -1)
    mm = m[c2]
    s = np.sqrt(np.maximum(1.0 + mm[:, 1, 1] - mm[:, 0, 0] - mm[:, 2, 2], 1e-300)) * 2
    q[c2] = np.stack([(mm[:, 0, 2] - mm[:, 2, 0]) / s, (mm[:, 0, 1] + mm[:, 1, 0]) / s,
                      0.25 * s, (mm[:, 1, 2] + mm[:, 2, 1]) / s], -1)
    mm = m[c3]
    s = np.sqrt(np.maximum(1.0 + mm[:, 2, 2] - mm[:, 0, 0] - mm[:, 1, 1], 1e-300)) * 2
    q[c3] = np.stack([(mm[:, 1, 0] - mm[:, 0, 1]) / s, (mm[:, 0, 2] + mm[:, 2, 0]) / s,
                      (mm[:, 1, 2] + mm[:, 2, 1]) / s, 0.25 * s], -1)
    return q


def _targets(rng, scene, depth_lo=None, depth_hi=None):
    n = scene.total_pixels
    scene.target_rgb = rng.random((3, n)).astype(np.float32)
    if depth_lo is not None:
        scene.target_depth = rng.uniform(depth_lo, depth_hi, n).astype(np.float32)
    return scene


# --------------------------------------------------------------------------
# the five workloads and the headline batch
# --------------------------------------------------------------------------

def config0():
    """One 64x48 view, 2,000 surfels in [-1,1]^2 x [2,6], L1 RGB loss."""
    seed = SEED_BASE + 0
    rng = np.random.Generator(np.random.PCG64(seed))
    sm = _surfels(rng, 2000, [-1, -1, 2], [1, 1, 6])
    vm = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
    sc = Scene("config0_64x48_2k", [sm], [(64, 48, 0)],
               np.array([[60, 60, 32, 24]], np.float32), vm, w_rgb=1.0, w_depth=0.0)
    return _targets(np.random.Generator(np.random.PCG64(seed + 1000)), sc)


def config1(n=300_000):
    """One 640x480 view (fx=fy=525), 300k surfels in [-3,3]^2 x [1,8],
    L1 RGB + 0.1 L1 depth against U[0,1] / U[1,8] targets."""
    seed = SEED_BASE + 1
    rng = np.random.Generator(np.random.PCG64(seed))
    sm = _surfels(rng, n, [-3, -3, 1], [3, 3, 8])
    vm = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
    sc = Scene("config1_640x480_300k", [sm], [(640, 480, 0)],
               np.array([[525, 525, 320, 240]], np.float32), vm, w_rgb=1.0, w_depth=0.1)
    return _targets(np.random.Generator(np.random.PCG64(seed + 1000)), sc, 1.0, 8.0)


def config2(n=1_000_000, n_views=16):
    """16 keyframes at 512x384 (fx=fy=420) over one shared 1M-surfel map."""
    seed = SEED_BASE + 2
    rng = np.random.Generator(np.random.PCG64(seed))
    sm = _surfels(rng, n, [-3, -3, 1], [3, 3, 8])
    vms = trajectory(rng, n_views).astype(np.float32)
    intr = np.tile(np.array([[420, 420, 256, 192]], np.float32), (n_views, 1))
    sc = Scene(f"config2_{n_views}x512x384_1M", [sm], [(512, 384, 0)] * n_views, intr, vms,
               w_rgb=1.0, w_depth=0.1)
    return _targets(np.random.Generator(np.random.PCG64(seed + 1000)), sc, 1.0, 8.0)


def headline(n_views=16):
    """The 640x480 headline batch: config 1's 300k-surfel scene seen from 16
    poses of the smooth random trajectory."""
    base = config1()
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 5))
    vms = trajectory(rng, n_views).astype(np.float32)
    intr = np.tile(np.array([[525, 525, 320, 240]], np.float32), (n_views, 1))
    sc = Scene(f"headline_{n_views}x640x480_300k", base.submaps, [(640, 480, 0)] * n_views,
               intr, vms, w_rgb=1.0, w_depth=0.1)
    return _targets(np.random.Generator(np.random.PCG64(SEED_BASE + 5 + 1000)), sc, 1.0, 8.0)


def config3(n_views=64, n_submaps=8, size_cap=None):
    """Uneven batch: 64 views over 8 submaps of log-uniform size in
    [50k, 2M]; view sizes uniform over {320x240, 640x480, 1280x720};
    fx=fy=525*W/640, principal point at the image centre; view j shows
    submap j mod 8 along that submap's own trajectory."""
    seed = SEED_BASE + 3
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.round(np.exp(rng.uniform(math.log(5e4), math.log(2e6), n_submaps))).astype(np.int64)
    if size_cap is not None:
        sizes = np.minimum(sizes, size_cap)
    subs = [_surfels(rng, int(s), [-3, -3, 1], [3, 3, 8]) for s in sizes]
    choices = [(320, 240), (640, 480), (1280, 720)]
    pick = rng.integers(0, 3, n_views)
    per_sub = [trajectory(rng, (n_views + n_submaps - 1 - j) // n_submaps) for j in range(n_submaps)]
    used = [0] * n_submaps
    views, intr, vms = [], [], []
    for j in range(n_views):
        w, h = choices[pick[j]]
        s = j % n_submaps
        views.append((w, h, s))
        f = 525.0 * w / 640.0
        intr.append([f, f, w / 2.0, h / 2.0])
        vms.append(per_sub[s][used[s]])
        used[s] += 1
    sc = Scene(f"config3_{n_views}views_{n_submaps}submaps", subs, views,
               np.asarray(intr, np.float32), np.asarray(vms, np.float32), w_rgb=1.0, w_depth=0.1,
               meta=dict(submap_sizes=[int(s) for s in sizes]))
    return _targets(np.random.Generator(np.random.PCG64(seed + 1000)), sc, 1.0, 8.0)


def _depth_field(rng, w, h, n_waves=6, lo=1.0, hi=6.0):
    yy, xx = np.meshgrid(np.arange(h) / h, np.arange(w) / w, indexing="ij")
    d = np.zeros((h, w))
    for _ in range(n_waves):
        fx, fy = rng.uniform(-2.0, 2.0, 2)
        ph = rng.uniform(0, 2 * math.pi)
        amp = rng.uniform(0.5, 1.0)
        d += amp * np.sin(2 * math.pi * (fx * xx + fy * yy) + ph)
    d = (d - d.min()) / max(d.max() - d.min(), 1e-12)
    return lo + (hi - lo) * d


def per_pixel_camera(rng, w, h, fx, fy, cx, cy):
    """One frame of a pixel-aligned surfel map in camera coordinates, as
    (centres [h,w,3], tangent frames [h,w,3,3] with columns t_u, t_v, n,
    scales [2,h*w], opacity [h*w], colour [3,h*w]): a smooth random depth
    field in [1,6], centres unprojected through the pixel centres, normals
    from central-difference tangents (facing the camera), tangent frame
    t_u = normalise(e_x - (e_x.n)n), t_v = n x t_u, scales depth/fx *
    U(0.5,1.5), opacity U(0.3,1), colour U[0,1]."""
    d = _depth_field(rng, w, h)
    yy, xx = np.meshgrid(np.arange(h) + 0.5, np.arange(w) + 0.5, indexing="ij")
    mu = np.stack([(xx - cx) / fx * d, (yy - cy) / fy * d, d], -1)          # [h,w,3] camera
    gx = np.gradient(mu, axis=1)
    gy = np.gradient(mu, axis=0)
    n = np.cross(gx, gy)
    n /= np.maximum(np.linalg.norm(n, axis=-1, keepdims=True), 1e-12)
    flip = np.sum(n * mu, -1) > 0
    n[flip] *= -1.0
    ex = np.array([1.0, 0.0, 0.0])
    tu = ex - np.sum(n * ex, -1, keepdims=True) * n
    tu /= np.maximum(np.linalg.norm(tu, axis=-1, keepdims=True), 1e-12)
    tv = np.cross(n, tu)
    rs = np.stack([tu, tv, n], -1)                                         # columns
    npx = w * h
    scale = (d.reshape(1, -1) / fx) * rng.uniform(0.5, 1.5, (2, npx))
    opacity = rng.uniform(0.3, 1.0, npx)
    color = rng.random((3, npx))
    return mu, rs, scale, opacity, color


def _planes(mu, rs, scale, opacity, color):
    q = quat_from_matrix(rs.reshape(-1, 3, 3))
    return dict(mean=np.ascontiguousarray(mu.reshape(-1, 3).T.astype(np.float32)),
                quat=np.ascontiguousarray(q.T.astype(np.float32)),
                scale=np.ascontiguousarray(scale.astype(np.float32)),
                opacity=opacity.astype(np.float32),
                color=color.astype(np.float32))


def per_pixel_frame(rng, w, h, fx, fy, cx, cy, r_wc, c):
    """per_pixel_camera's map moved into world coordinates by the camera
    rotation r_wc and centre c."""
    mu, rs, scale, opacity, color = per_pixel_camera(rng, w, h, fx, fy, cx, cy)
    return _planes(mu @ r_wc.T + c, np.einsum("ij,hwjk->hwik", r_wc, rs), scale, opacity, color)


@dataclass
class FusionFrame:
    """A frame for map fusion: its per-pixel map in camera coordinates, its
    camera-to-world similarity x_w = s R(q) x_c + t and an accumulated-alpha
    map of the global map rendered from it."""
    width: int
    height: int
    planes: dict
    s: float
    q: np.ndarray
    t: np.ndarray
    accum: np.ndarray


def fusion_frames(n_frames=32, w=518, h=392, seed_offset=0):
    """Frames of the map-fusion workload: config-4 per-pixel maps in camera
    coordinates, poses along config 4's small-step trajectory with a scale in
    U(0.9, 1.1), and accumulation maps from a smooth random field in [0, 1]."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 40 + seed_offset))
    fx = fy = 400.0
    cx, cy = w / 2.0, h / 2.0
    out = []
    pos = np.zeros(3)
    yaw = 0.0
    for _ in range(n_frames):
        yaw += math.radians(rng.uniform(-1.0, 1.0))
        pos = pos + rng.uniform(-0.02, 0.02, 3)
        planes = _planes(*per_pixel_camera(rng, w, h, fx, fy, cx, cy))
        q = quat_from_matrix(_rot_y(yaw).reshape(1, 3, 3))[0]
        acc = (_depth_field(rng, w, h, lo=0.0, hi=1.0)).reshape(-1)
        out.append(FusionFrame(w, h, planes, float(rng.uniform(0.9, 1.1)), q.astype(np.float32),
                               pos.astype(np.float32), acc.astype(np.float32)))
    return out


def config4(n_frames=32, stress=False, w=518, h=392):
    """Per-pixel surfel maps of the kind the feed-forward frontend emits:
    32 frames at 518x392 (fx=fy=400, cx=259, cy=196), one surfel per pixel.
    Render pose k = frame pose k composed with a seeded perturbation
    (<= 1 deg, <= 0.03).  Default: view k renders frame k's surfels (the
    per-frame loss); stress: every view renders all frames' surfels."""
    seed = SEED_BASE + 4
    rng = np.random.Generator(np.random.PCG64(seed))
    fx = fy = 400.0
    cx, cy = w / 2.0, h / 2.0
    frames, vms = [], []
    pos = np.zeros(3)
    yaw = 0.0
    for k in range(n_frames):
        yaw += math.radians(rng.uniform(-1.0, 1.0))
        pos = pos + rng.uniform(-0.02, 0.02, 3)
        r_wc = _rot_y(yaw)
        frames.append(per_pixel_frame(rng, w, h, fx, fy, cx, cy, r_wc, pos))
        ax = rng.standard_normal(3)
        ang = math.radians(rng.uniform(0.0, 1.0))
        d = rng.standard_normal(3)
        d *= rng.uniform(0.0, 0.03) / np.linalg.norm(d)
        r_p = r_wc @ _rot_axis(ax, ang)
        vms.append(_viewmat_from_cam(r_p, pos + r_wc @ d))
    intr = np.tile(np.array([[fx, fy, cx, cy]], np.float32), (n_frames, 1))
    if stress:
        cat = {k: np.concatenate([f[k] for f in frames], axis=-1) for k in frames[0]}
        subs = [cat]
        views = [(w, h, 0)] * n_frames
    else:
        subs = frames
        views = [(w, h, k) for k in range(n_frames)]
    sc = Scene(f"config4_{n_frames}x{w}x{h}_perpixel" + ("_stress" if stress else ""), subs, views,
               intr, np.asarray(vms, np.float32), w_rgb=1.0, w_depth=0.1)
    return _targets(np.random.Generator(np.random.PCG64(seed + 1000)), sc, 1.0, 6.0)


def random_scene(seed, n, w, h, n_views=1, fx=None, lo=(-1, -1, 2), hi=(1, 1, 6),
                 scale_lo=0.01, scale_hi=0.1, depth_target=True):
    """Small scene for tests: config-0 laws at a chosen size and view count."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sm = _surfels(rng, n, lo, hi, scale_lo, scale_hi)
    f = float(fx if fx is not None else w * 60.0 / 64.0)
    if n_views == 1:
        vms = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
    else:
        vms = (trajectory(rng, n_views) * np.array([1, 1, 1, 0.3] * 3)).astype(np.float32)
    intr = np.tile(np.array([[f, f, w / 2.0, h / 2.0]], np.float32), (n_views, 1))
    sc = Scene(f"random_{seed}_{n}_{w}x{h}x{n_views}", [sm], [(w, h, 0)] * n_views, intr, vms,
               w_rgb=1.0, w_depth=0.1 if depth_target else 0.0)
    return _targets(np.random.Generator(np.random.PCG64(seed + 1000)), sc,
                    *((1.0, 8.0) if depth_target else (None, None)))


def largest_view_clusters(seed=SEED_BASE + 41, size=16384, f=8000.0, n_per=600, crop=512, spread=100.0):
    """One view at the largest supported size with surfels in two small
    clusters, near the top-left and the bottom-right corner.  Each cluster's
    centres lie on rays within `spread` pixels of its centre pixel at depths
    in [3, 5], with tangent scales log-uniform in [0.002, 0.006] (supports
    under 50 pixels), so every support stays inside the crop x crop window
    whose corner (x0, y0) is listed in meta["crops"]; the rest of the image
    is empty.  No targets."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = size / 2.0
    parts, crops = [], []
    for (px, py) in [(300.0, 260.0), (size - 300.0, size - 260.0)]:
        sm = _surfels(rng, n_per, (0, 0, 3), (1, 1, 5), 0.002, 0.006)
        z = sm["mean"][2].astype(np.float64)
        u = px + rng.uniform(-spread, spread, n_per)
        v = py + rng.uniform(-spread, spread, n_per)
        sm["mean"] = np.ascontiguousarray(np.stack([(u - c) * z / f, (v - c) * z / f, z]).astype(np.float32))
        parts.append(sm)
        crops.append((int(px) - crop // 2, int(py) - crop // 2))
    sm = {k: np.ascontiguousarray(np.concatenate([p[k] for p in parts], axis=-1)) for k in parts[0]}
    intr = np.array([[f, f, c, c]], np.float32)
    vm = np.array([[1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]], np.float32)
    return Scene(f"largest_view_{size}x{size}", [sm], [(size, size, 0)], intr, vm,
                 meta=dict(crops=crops, crop=crop))


def make(name):
    """Scene by name: config0..config4, config4_stress, headline."""
    table = {"config0": config0, "config1": config1, "config2": config2,
             "config3": config3, "config4": config4, "headline": headline,
             "config4_stress": lambda: config4(stress=True)}
    return table[name]()
