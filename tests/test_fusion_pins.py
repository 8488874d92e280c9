"""Pins of the map-fusion oracle (CPU): hand-built blocks with closed-form
means, sign-aligned quaternion averaging, the border blocks, the order of the
output, the accumulation gate, and the similarity transform against scipy's
rotation conventions."""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle import fusion
from paper_2604_03092_amd import scenes

ID_Q = np.array([1.0, 0.0, 0.0, 0.0])


def _map(W, H, rng, z=None):
    P = W * H
    q = rng.normal(size=(4, P))
    q /= np.linalg.norm(q, axis=0)
    return dict(mean=np.stack([rng.uniform(-1, 1, P), rng.uniform(-1, 1, P),
                               z if z is not None else rng.uniform(1, 6, P)]).astype(np.float32),
                quat=q.astype(np.float32), scale=rng.uniform(0.01, 0.1, (2, P)).astype(np.float32),
                opacity=rng.uniform(0.3, 1, P).astype(np.float32),
                color=np.arange(3 * P, dtype=np.float32).reshape(3, P) / (3 * P))


def test_no_merge_identity_pose_is_identity():
    rng = np.random.default_rng(1)
    pl = _map(5, 3, rng)
    out = fusion.voxelize_fuse(5, 3, pl, 1.0, ID_Q, np.zeros(3), tau_depth=-1.0)
    # blocks in row-major order, pixels row-major inside a block
    order = [0, 1, 5, 6, 2, 3, 7, 8, 4, 9, 10, 11, 12, 13, 14]
    for k in pl:
        np.testing.assert_array_equal(out[k], pl[k][..., order].astype(np.float64))


def test_merge_means_and_border_blocks():
    rng = np.random.default_rng(2)
    pl = _map(3, 3, rng, z=np.full(9, 2.0))
    out = fusion.voxelize_fuse(3, 3, pl, 1.0, ID_Q, np.zeros(3), tau_depth=0.5)
    # blocks: {0,1,3,4}, {2,5}, {6,7}, {8}
    groups = [[0, 1, 3, 4], [2, 5], [6, 7], [8]]
    assert out["opacity"].shape == (4,)
    for j, g in enumerate(groups):
        for k in ("mean", "scale", "color"):
            np.testing.assert_allclose(out[k][:, j], pl[k][:, g].astype(np.float64).mean(1), rtol=1e-12)
        np.testing.assert_allclose(out["opacity"][j], pl["opacity"][g].astype(np.float64).mean(), rtol=1e-12)
    # the single-pixel block is passed through untouched (no renormalisation)
    np.testing.assert_array_equal(out["quat"][:, 3], pl["quat"][:, 8].astype(np.float64))


def test_depth_range_splits_blocks():
    rng = np.random.default_rng(3)
    z = np.array([2.0, 2.05, 3.0, 2.02, 2.0, 3.5], np.float32)   # 3x2: blocks {0,1,3,4}, {2,5}
    pl = _map(3, 2, rng, z=z)
    out = fusion.voxelize_fuse(3, 2, pl, 1.0, ID_Q, np.zeros(3), tau_depth=0.1)
    # first block's range 0.05 <= 0.1: merged; second 0.5 > 0.1: kept as 2
    assert out["opacity"].shape == (3,)
    np.testing.assert_allclose(out["mean"][:, 0], pl["mean"][:, [0, 1, 3, 4]].astype(np.float64).mean(1))
    np.testing.assert_array_equal(out["mean"][:, 1:], pl["mean"][:, [2, 5]].astype(np.float64))


def test_quaternion_sign_alignment():
    rng = np.random.default_rng(4)
    pl = _map(2, 2, rng, z=np.full(4, 3.0))
    base = Rotation.from_rotvec([0.3, -0.2, 0.1])
    small = [Rotation.from_rotvec(rng.normal(0, 0.05, 3)) for _ in range(4)]
    qs = np.stack([(base * r).as_quat() for r in small])      # scipy (x, y, z, w)
    pl["quat"] = np.roll(qs, 1, axis=1).T.astype(np.float32)   # (w, x, y, z)
    a = fusion.voxelize_fuse(2, 2, pl, 1.0, ID_Q, np.zeros(3), tau_depth=1.0)
    flipped = dict(pl)
    flipped["quat"] = pl["quat"] * np.array([1, -1, 1, -1], np.float32)
    b = fusion.voxelize_fuse(2, 2, flipped, 1.0, ID_Q, np.zeros(3), tau_depth=1.0)
    np.testing.assert_allclose(a["quat"], b["quat"], atol=1e-7)
    # the merged rotation is close to the common base rotation
    r = Rotation.from_quat(np.roll(a["quat"][:, 0], -1))
    assert (r * base.inv()).magnitude() < 0.1


def test_similarity_transform_against_scipy():
    rng = np.random.default_rng(5)
    pl = _map(4, 4, rng)
    s, t = 1.07, np.array([0.3, -0.2, 0.9])
    rq = Rotation.from_rotvec([0.2, 0.4, -0.3])
    q = np.roll(rq.as_quat(), 1)
    out = fusion.voxelize_fuse(4, 4, pl, s, q, t, tau_depth=-1.0)
    ref = fusion.voxelize_fuse(4, 4, pl, 1.0, ID_Q, np.zeros(3), tau_depth=-1.0)
    np.testing.assert_allclose(out["mean"], s * rq.apply(ref["mean"].T).T + t[:, None], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(out["scale"], s * ref["scale"], rtol=1e-12)
    r_out = Rotation.from_quat(np.roll(out["quat"].T, -1, axis=1))
    r_ref = rq * Rotation.from_quat(np.roll(ref["quat"].T, -1, axis=1))
    np.testing.assert_allclose(r_out.as_matrix(), r_ref.as_matrix(), atol=1e-12)


def test_accumulation_gate():
    rng = np.random.default_rng(6)
    pl = _map(4, 2, rng, z=np.full(8, 2.0))
    none = fusion.voxelize_fuse(4, 2, pl, 1.0, ID_Q, np.zeros(3), tau_depth=1.0)
    zeros = fusion.voxelize_fuse(4, 2, pl, 1.0, ID_Q, np.zeros(3), 1.0, np.zeros(8, np.float32), 0.5)
    ones = fusion.voxelize_fuse(4, 2, pl, 1.0, ID_Q, np.zeros(3), 1.0, np.ones(8, np.float32), 0.5)
    for k in none:
        np.testing.assert_array_equal(zeros[k], none[k])
    assert ones["opacity"].size == 0
    # blocks {0,1,4,5} (mean 0.45 < 0.5: added) and {2,3,6,7} (mean 0.55: not added)
    acc = np.array([0.1, 0.8, 0.2, 0.9, 0.4, 0.5, 0.6, 0.5], np.float32)
    mixed = fusion.voxelize_fuse(4, 2, pl, 1.0, ID_Q, np.zeros(3), 1.0, acc, 0.5)
    assert mixed["opacity"].size == 1
    np.testing.assert_allclose(mixed["mean"][:, 0], none["mean"][:, 0])
    # unmerged pixels are gated one by one
    kept = fusion.voxelize_fuse(4, 2, pl, 1.0, ID_Q, np.zeros(3), -1.0, acc, 0.5)
    assert kept["opacity"].size == int(np.sum(acc < 0.5))


def test_fusion_frames_generator():
    fr = scenes.fusion_frames(2, 9, 7)
    assert len(fr) == 2 and fr[0].planes["mean"].shape == (3, 63) and fr[0].accum.shape == (63,)
    assert 0.9 <= fr[0].s <= 1.1 and abs(np.linalg.norm(fr[0].q) - 1) < 1e-6
