"""Shared helpers of the GPU parity tests: oracle comparison and tolerances.

Tolerances (from the float32 arithmetic of the GPU path):
  * pair lists and tile ranges: exact, up to tiles of a surfel's bbox that
    its support does not reach (assert_pairs_match);
  * image planes: max-abs 1e-4 on pixels the oracle does not flag (a flag
    marks a pixel where some decision lies within the margin of its
    threshold or where the ray meets a surfel at a grazing angle);
  * gradients: relative L2 <= 1e-3 and, per element,
    |gpu - ref| <= 1e-3 (|ref| + rms(ref)).
"""
import numpy as np

IMG_ATOL = 1e-4
GRAD_REL = 1e-3


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def assert_images_close(out, ref, mask, atol=IMG_ATOL, what=""):
    for k in ("rgb", "depth", "normal", "alpha"):
        got = to_np(out[k])
        exp = ref[k]
        d = np.abs(got - exp)[..., mask]
        worst = float(d.max()) if d.size else 0.0
        assert worst <= atol, f"{what} {k}: max abs diff {worst:.3e} on unflagged pixels"


def grad_errors(got, ref):
    """(relative L2 error, worst per-element |got - ref| / (|ref| + rms(ref)))."""
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    nr = np.linalg.norm(ref)
    if nr == 0.0:
        return (0.0 if not np.abs(got).any() else np.inf), (0.0 if not np.abs(got).any() else np.inf)
    rms = np.sqrt(np.mean(ref ** 2))
    return float(np.linalg.norm(got - ref) / nr), float(np.max(np.abs(got - ref) / (np.abs(ref) + rms)))


def assert_grad_close(got, ref, name, rel=GRAD_REL):
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    nr = np.linalg.norm(ref)
    if nr == 0.0:
        assert np.abs(got).max() == 0.0, name
        return
    rl2 = np.linalg.norm(got - ref) / nr
    rms = np.sqrt(np.mean(ref ** 2))
    bad = np.abs(got - ref) > rel * (np.abs(ref) + rms)
    assert rl2 <= rel, f"{name}: relative L2 error {rl2:.3e}"
    assert not bad.any(), (f"{name}: {int(bad.sum())} elements out of tolerance, worst "
                           f"{float(np.max(np.abs(got - ref) / (np.abs(ref) + rms))):.3e}")


def random_upstream(rng, npx, keep):
    k = keep.astype(np.float64)
    return dict(rgb=rng.normal(size=(3, npx)) * k, depth=rng.normal(size=npx) * k,
                normal=rng.normal(size=(3, npx)) * k, alpha=rng.normal(size=npx) * k)


def assert_pairs_match(b, t, s, ts, te):
    """The GPU pair list of one view against the oracle's binning (bin_view).
    The pairs are unique up to tiles that the surfel's bbox spans but its
    support does not reach: the GPU list must be a sub-list of the oracle's
    bbox list, in the same (tile, depth key, index) order, that holds every
    pair whose surfel reaches a pixel of the tile (the oracle's
    pair_reached flags, every pair checked); the tile ranges must count the
    kept pairs.  Returns the fraction of the oracle's pairs kept."""
    n = 1 << 32
    ko = b["pair_tile"].astype(np.int64) * n + b["pair_surf"].astype(np.int64)
    kg = np.asarray(t, np.int64) * n + np.asarray(s, np.int64)
    keep = np.isin(ko, kg)
    assert np.array_equal(ko[keep], kg), "GPU pairs are not an ordered sub-list of the oracle's"
    missing = b["pair_reached"] & ~keep
    assert not missing.any(), f"{int(missing.sum())} pairs whose surfel reaches a pixel of the tile are missing"
    cnt = np.bincount(b["pair_tile"][keep].astype(np.int64), minlength=len(ts))
    assert np.array_equal((np.asarray(te) - np.asarray(ts)).astype(np.int64), cnt[:len(ts)])
    return float(keep.mean()) if keep.size else 1.0
