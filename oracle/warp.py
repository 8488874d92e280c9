"""FP64 oracle of the loop-correction warp (test infrastructure only).

Sec. 3.3 ("Loop Correction of Gaussian Map"): primitives stay bound to the
keyframe that created them; when loop closure moves a keyframe from T_old
to T_new, every primitive bound to it is moved rigidly by
Delta T = T_new T_old^-1.  For a similarity Delta T = (s, q, t): the centre
goes to s R(q) mu + t, the rotation to q r, and the tangent scales are
multiplied by s (as in map fusion).  Primitives whose keyframe index is out
of range (e.g. -1) are left alone.  Written from the definition with numpy;
shares nothing with the HIP path.
"""
from __future__ import annotations

import numpy as np


def quat_mul(a, b):
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz, aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx, aw * bz + ax * by - ay * bx + az * bw])


def rot(q):
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def compose(a, b):
    """Similarity a * b as (s, q, t): x -> a(b(x))."""
    sa, qa, ta = a
    sb, qb, tb = b
    qa = np.asarray(qa, np.float64) / np.linalg.norm(qa)
    qb = np.asarray(qb, np.float64) / np.linalg.norm(qb)
    return sa * sb, quat_mul(qa, qb), sa * rot(qa) @ np.asarray(tb, np.float64) + np.asarray(ta, np.float64)


def inverse(a):
    s, q, t = a
    q = np.asarray(q, np.float64) / np.linalg.norm(q)
    qi = q * np.array([1, -1, -1, -1])
    return 1.0 / s, qi, -(rot(qi) @ np.asarray(t, np.float64)) / s


def warp(planes, keyframe, deltas):
    """planes: dict of SoA arrays (mean [3,n], quat [4,n], scale [2,n]);
    keyframe: int [n]; deltas: list of (s, q, t).  Returns new float64 planes."""
    mean = planes["mean"].astype(np.float64).copy()
    quat = planes["quat"].astype(np.float64).copy()
    scale = planes["scale"].astype(np.float64).copy()
    for i, k in enumerate(keyframe):
        if not 0 <= k < len(deltas):
            continue
        s, q, t = deltas[k]
        q = np.asarray(q, np.float64) / np.linalg.norm(q)
        mean[:, i] = s * rot(q) @ mean[:, i] + np.asarray(t, np.float64)
        quat[:, i] = quat_mul(q, quat[:, i])
        scale[:, i] = s * scale[:, i]
    return dict(mean=mean, quat=quat, scale=scale)
