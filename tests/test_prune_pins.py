"""Pins of the oracle's map-fusion pruning (Sec. 3.3, "Map Fusion"): the
error criterion on hand-built pixels, the contribution score against closed
forms of Eq. 1 and against the backward's colour gradient (a separate
reverse-sweep code path), and the removal on a hand-built score list."""
import math

import numpy as np
import pytest

from oracle import prune
from paper_2604_03092_amd import scenes

A_MIN = float(np.float32(1.0 / 255.0))
IDENT = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)


def one_surfel(mu, quat, scale, sigma, color):
    f = lambda a: np.asarray(a, np.float32).reshape(-1, 1)
    return dict(mean=f(mu), quat=f(quat), scale=f(scale), opacity=np.asarray([sigma], np.float32),
                color=f(color))


def stack(*sms):
    return {k: np.concatenate([s[k] for s in sms], axis=-1) for k in sms[0]}


def test_error_mask_hand_built():
    # pixel 0: mean error (0.3 + 0 + 0)/3 = 0.1; pixel 1: 0.04; pixel 2: rgb exact, depth off by 0.5
    rgb = np.array([[0.5, 0.54, 0.2], [0.5, 0.5, 0.3], [0.5, 0.5, 0.4]])
    tgt = np.array([[0.2, 0.5, 0.2], [0.5, 0.42, 0.3], [0.5, 0.5, 0.4]])
    depth = np.array([2.0, 3.0, 4.5])
    tdep = np.array([2.0, 3.0, 4.0])
    assert list(prune.error_mask(rgb, depth, tgt, None, 0.05)) == [True, False, False]
    assert list(prune.error_mask(rgb, depth, tgt, None, 0.03)) == [True, True, False]
    assert list(prune.error_mask(rgb, depth, tgt, tdep, 0.05, 0.25)) == [True, False, True]
    assert list(prune.error_mask(rgb, depth, tgt, tdep, 0.2, 0.6)) == [False, False, False]
    for tau in (0.03, 0.05, 0.2):
        assert np.array_equal(prune.error_mask_f32(rgb, depth, tgt, tdep, tau, 0.25),
                              prune.error_mask(rgb, depth, tgt, tdep, tau, 0.25))


def test_error_mask_f32_agrees_away_from_the_threshold():
    rng = np.random.default_rng(3)
    rgb, tgt = rng.random((3, 20000)), rng.random((3, 20000))
    d, td = rng.uniform(1, 8, 20000), rng.uniform(1, 8, 20000)
    tau, tau_d = 0.3, 2.0
    a = prune.error_mask(rgb.astype(np.float32), d.astype(np.float32), tgt.astype(np.float32),
                         td.astype(np.float32), tau, tau_d)
    b = prune.error_mask_f32(rgb, d, tgt, td, tau, tau_d)
    e = np.mean(np.abs(rgb.astype(np.float32).astype(np.float64) - tgt.astype(np.float32)), axis=0)
    near = np.abs(e - tau) < 1e-6
    assert np.array_equal(a[~near], b[~near])
    assert 0.1 < a.mean() < 0.9


def test_score_single_surfel_closed_form():
    """One fronto-parallel surfel at the identity pose, every pixel masked:
    its score is the sum over pixels of alpha = min(0.99, sigma exp(-r^2/2))
    with u = (x - cx - fx X/Z) Z/(fx s_u), v likewise (T = 1 everywhere)."""
    w, h = 40, 32
    intr = np.array([50, 55, 20.5, 15.0], np.float32)
    X, Y, Z, su, sv, sig = 0.1, -0.05, 3.0, 0.2, 0.12, 0.8
    sm = one_surfel([X, Y, Z], [1, 0, 0, 0], [su, sv], sig, [0.3, 0.6, 0.9])
    s = prune.contribution_scores_view(sm, w, h, intr, IDENT, np.ones(w * h, bool))
    yy, xx = np.meshgrid(np.arange(h) + 0.5, np.arange(w) + 0.5, indexing="ij")
    fx, fy, cx, cy = [float(v) for v in intr]
    X, Y, Z, su, sv, sig = [float(np.float32(v)) for v in (X, Y, Z, su, sv, sig)]
    u = (xx - cx - fx * X / Z) * Z / (fx * su)
    v = (yy - cy - fy * Y / Z) * Z / (fy * sv)
    r2 = u * u + v * v
    at = sig * np.exp(-0.5 * r2)
    a = np.where((r2 <= 9.0) & (at >= A_MIN), np.minimum(at, float(np.float32(0.99))), 0.0)
    np.testing.assert_allclose(s[0], a.sum(), rtol=1e-12)
    # half the pixels masked: only those count
    half = (xx < 20).reshape(-1)
    s2 = prune.contribution_scores_view(sm, w, h, intr, IDENT, half)
    np.testing.assert_allclose(s2[0], a[xx < 20].sum(), rtol=1e-12)


def test_score_stack_closed_form():
    """Two fronto-parallel surfels centred on pixel (8, 8), one masked pixel:
    the front one scores alpha_1, the back one alpha_2 (1 - alpha_1)."""
    intr = np.array([20, 20, 8.5, 8.5], np.float32)
    sm = stack(one_surfel([0, 0, 3.0], [1, 0, 0, 0], [0.5, 0.5], 0.7, [0, 0, 0]),
               one_surfel([0, 0, 2.0], [1, 0, 0, 0], [0.5, 0.5], 0.4, [0, 0, 0]))
    mask = np.zeros(256, bool)
    mask[8 * 16 + 8] = True
    s = prune.contribution_scores_view(sm, 16, 16, intr, IDENT, mask)
    a_front, a_back = float(np.float32(0.4)), float(np.float32(0.7))
    np.testing.assert_allclose(s, [a_back * (1 - a_front), a_front], rtol=1e-12)


def test_score_equals_colour_gradient_of_the_masked_red_channel(orc):
    """Eq. 1 is linear in the colours: dI_r/dc_{k,r} = alpha_k T_k, so with
    the upstream gradient (mask, 0, 0) on the image the backward's red
    colour gradient (the reverse-sweep code path) is the score."""
    sc = scenes.random_scene(81, 3000, 64, 48, n_views=2, scale_lo=0.03, scale_hi=0.2)
    rng = np.random.default_rng(82)
    mask = rng.random(sc.total_pixels) < 0.3
    s = prune.contribution_scores(sc, mask)
    P = sc.total_pixels
    g = dict(rgb=np.stack([mask.astype(np.float64), np.zeros(P), np.zeros(P)]), depth=np.zeros(P),
             normal=np.zeros((3, P)), alpha=np.zeros(P))
    grads, _ = orc.backward_scene(sc, g)
    np.testing.assert_allclose(s[0], grads[0]["color"][0], rtol=1e-10, atol=1e-14)
    assert (s[0] > 0).mean() > 0.1


def test_prune_keep_hand_built():
    score = np.array([0.0, 0.5, 0.2, 0.0, 1e-9, 0.2], np.float32)
    assert list(prune.prune_keep(score, 0.0)) == [0, 3]
    assert list(prune.prune_keep(score, 0.2)) == [0, 2, 3, 4, 5]
    assert list(prune.prune_keep(score, 1.0)) == [0, 1, 2, 3, 4, 5]
    sm = {"opacity": np.arange(6, dtype=np.float32), "mean": np.arange(18, dtype=np.float32).reshape(3, 6)}
    out = prune.prune_surfels(sm, score, 0.2)
    assert list(out["opacity"]) == [0, 2, 3, 4, 5]
    assert out["mean"].shape == (3, 5) and list(out["mean"][2]) == [12, 14, 15, 16, 17]
