"""Pins of the loop-correction warp oracle (CPU): identity, round trip with
the inverse, composition, agreement with scipy's rotations, and untouched
unbound primitives."""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle import warp


def _planes(n, rng):
    q = rng.normal(size=(4, n))
    return dict(mean=rng.normal(size=(3, n)).astype(np.float32), quat=(q / np.linalg.norm(q, axis=0)).astype(np.float32),
                scale=rng.uniform(0.01, 0.1, (2, n)).astype(np.float32))


def _sim(rng):
    r = Rotation.from_rotvec(rng.normal(0, 0.5, 3))
    return float(rng.uniform(0.8, 1.2)), np.roll(r.as_quat(), 1), rng.normal(0, 1, 3)


def test_identity_and_unbound():
    rng = np.random.default_rng(0)
    pl = _planes(50, rng)
    kf = rng.integers(-1, 3, 50)
    ident = [(1.0, np.array([1.0, 0, 0, 0]), np.zeros(3))] * 3
    out = warp.warp(pl, kf, ident)
    for k in out:
        np.testing.assert_array_equal(out[k], pl[k].astype(np.float64))
    moved = warp.warp(pl, kf, [_sim(rng) for _ in range(3)])
    for k in out:
        np.testing.assert_array_equal(moved[k][:, kf < 0], pl[k][:, kf < 0].astype(np.float64))


def test_round_trip_and_composition():
    rng = np.random.default_rng(1)
    pl = _planes(40, rng)
    kf = rng.integers(0, 4, 40)
    d = [_sim(rng) for _ in range(4)]
    back = warp.warp(warp.warp(pl, kf, d), kf, [warp.inverse(x) for x in d])
    for k in back:
        np.testing.assert_allclose(back[k] * np.sign(back["quat"][0] if k == "quat" else 1),
                                   pl[k] * np.sign(pl["quat"][0] if k == "quat" else 1), atol=1e-12)
    e = [_sim(rng) for _ in range(4)]
    two = warp.warp(warp.warp(pl, kf, d), kf, e)
    one = warp.warp(pl, kf, [warp.compose(b, a) for a, b in zip(d, e)])
    for k in one:
        np.testing.assert_allclose(two[k], one[k], atol=1e-12)


def test_against_scipy():
    rng = np.random.default_rng(2)
    pl = _planes(30, rng)
    kf = np.zeros(30, int)
    s, q, t = _sim(rng)
    out = warp.warp(pl, kf, [(s, q, t)])
    r = Rotation.from_quat(np.roll(q, -1))
    np.testing.assert_allclose(out["mean"], s * r.apply(pl["mean"].T.astype(np.float64)).T + t[:, None], atol=1e-12)
    got = Rotation.from_quat(np.roll(out["quat"].T, -1, axis=1)).as_matrix()
    ref = (r * Rotation.from_quat(np.roll(pl["quat"].T.astype(np.float64), -1, axis=1))).as_matrix()
    np.testing.assert_allclose(got, ref, atol=1e-12)
    np.testing.assert_allclose(out["scale"], s * pl["scale"].astype(np.float64), rtol=1e-15)
