"""FP64 oracle of map fusion for an incoming per-pixel surfel map (test
infrastructure only).

Adaptive voxelization (Sec. 3.3, "Adaptive Voxelization"): the pixel grid is
cut into 2x2 blocks; a block whose camera-space depth range (max z - min z)
is at most tau_depth is replaced by one primitive whose centre, opacity,
colour and scales are the means over the block and whose rotation is the
normalised sum of the block's quaternions, each first sign-aligned with the
block's first one (Eq. for r_merged).  Other blocks keep their primitives.
Blocks cut by the image border hold 2 or 1 pixels; a 1-pixel block is kept
as it is.  The surviving primitives are moved to world coordinates by the
frame's similarity, mu_w = s R mu + t and r_w = q * r (the map-fusion
transform), with the scales multiplied by s.  With an accumulation map of
the global map rendered from the frame, only primitives in regions that are
not yet well reconstructed are added: a kept pixel's own value, a merged
block's mean value, must be below tau_accum.

Where a float decides what is merged or kept, the decision is taken in
float32 with the operation order the GPU uses (as the API carries float32).
Output order: blocks in row-major order of the block grid; inside a kept
block its pixels in row-major order.  Written from the definitions with
numpy; shares nothing with the HIP path.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def _quat_mul(a, b):
    """Hamilton product of (w, x, y, z) quaternions, arrays [..., 4]."""
    aw, ax, ay, az = (a[..., i] for i in range(4))
    bw, bx, by, bz = (b[..., i] for i in range(4))
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], -1)


def _rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _align_sign(qn, q0):
    """-1 where the float32 dot product of qn with q0 is negative."""
    a = qn.astype(f32)
    b = q0.astype(f32)
    d = (a[0] * b[0] + a[1] * b[1]) + (a[2] * b[2] + a[3] * b[3])
    return -1.0 if d < f32(0) else 1.0


def voxelize_fuse(width, height, planes, s, q, t, tau_depth, accum=None, tau_accum=1.0):
    """planes: dict of float32 SoA arrays (mean [3,P], quat [4,P], scale [2,P],
    opacity [P], color [3,P]) in camera coordinates, P = width * height.
    Returns the fused primitives as float64 SoA arrays in world coordinates."""
    W, H = width, height
    mean = planes["mean"].astype(np.float64)
    quat = planes["quat"].astype(np.float64)
    scale = planes["scale"].astype(np.float64)
    opac = planes["opacity"].astype(np.float64)
    col = planes["color"].astype(np.float64)
    z32 = planes["mean"][2].astype(f32)
    a32 = None if accum is None else accum.astype(f32)
    tau_d = f32(tau_depth)
    tau_a = f32(tau_accum)
    out = {k: [] for k in ("mean", "quat", "scale", "opacity", "color")}

    def emit(mu, r, sc, o, c):
        out["mean"].append(mu)
        out["quat"].append(r)
        out["scale"].append(sc)
        out["opacity"].append(o)
        out["color"].append(c)

    for by in range((H + 1) // 2):
        for bx in range((W + 1) // 2):
            px = [(2 * by + dy) * W + 2 * bx + dx for dy in (0, 1) for dx in (0, 1)
                  if 2 * bx + dx < W and 2 * by + dy < H]
            n = len(px)
            zs = [z32[p] for p in px]
            merge = n > 1 and (max(zs) - min(zs)) <= tau_d
            if merge:
                if a32 is not None:
                    a = [a32[p] for p in px]
                    tot = (a[0] + a[1]) + (a[2] + a[3]) if n == 4 else a[0] + a[1]
                    if not tot < tau_a * f32(n):
                        continue
                r = sum(_align_sign(quat[:, p], quat[:, px[0]]) * quat[:, p] for p in px)
                emit(mean[:, px].mean(1), r / np.linalg.norm(r), scale[:, px].mean(1), opac[px].mean(),
                     col[:, px].mean(1))
            else:
                for p in px:
                    if a32 is not None and not a32[p] < tau_a:
                        continue
                    emit(mean[:, p], quat[:, p], scale[:, p], opac[p], col[:, p])
    n_out = len(out["opacity"])
    R = _rot(np.asarray(q, np.float64))
    qn = np.asarray(q, np.float64) / np.linalg.norm(q)
    res = {}
    if n_out == 0:
        return dict(mean=np.zeros((3, 0)), quat=np.zeros((4, 0)), scale=np.zeros((2, 0)), opacity=np.zeros(0),
                    color=np.zeros((3, 0)))
    mu = np.stack(out["mean"], 1)
    res["mean"] = s * (R @ mu) + np.asarray(t, np.float64)[:, None]
    res["quat"] = _quat_mul(qn[None, :], np.stack(out["quat"], 0)).T
    res["scale"] = s * np.stack(out["scale"], 1)
    res["opacity"] = np.asarray(out["opacity"])
    res["color"] = np.stack(out["color"], 1)
    return res
