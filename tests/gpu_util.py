"""Shared helpers of the GPU parity tests: oracle comparison and tolerances.

Tolerances (from the float32 arithmetic of the GPU path):
  * pair lists and tile ranges: exact;
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
