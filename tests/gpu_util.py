"""Shared helpers of the GPU parity tests: oracle comparison and tolerances.

Tolerances (from the float32 arithmetic of the GPU path):
  * pair lists and tile ranges: exact, up to the tiles the GPU leaves out
    (assert_pairs_match);
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


def _support_min_margin(sm, intr, viewmat, surf, tiles, tiles_x, tile_w, tile_h, width, height,
                        alpha_min=1.0 / 255.0, rho_max=3.0):
    """For each (surfel, tile): the smallest r^2 / rho_eff^2 over the tile's
    pixel centres, in FP64 from the definition (H = K [s_u t_u | s_v t_v | p],
    w = (H0 - x H2) x (H1 - y H2), r^2 = (w0^2 + w1^2) / w2^2,
    rho_eff^2 = min(rho_max^2, 2 ln(sigma / alpha_min))).  A value above 1
    means that no pixel of the tile is covered."""
    mean = np.asarray(sm["mean"], np.float64)[:, surf]
    q = np.asarray(sm["quat"], np.float64)[:, surf]
    sc = np.asarray(sm["scale"], np.float64)[:, surf]
    sig = np.asarray(sm["opacity"], np.float64)[surf]
    q = q / np.linalg.norm(q, axis=0)
    w, x, y, z = q
    # columns 0 and 1 of the rotation of q
    e1 = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)])
    e2 = np.stack([2 * (x * y - w * z), 1 - 2 * (x * x + z * z), 2 * (y * z + w * x)])
    vm = np.asarray(viewmat, np.float64).reshape(3, 4)
    R, t = vm[:, :3], vm[:, 3]
    fx, fy, cx, cy = np.asarray(intr, np.float64)
    K = np.array([[fx, 0, cx], [0, fy, cy], [0, 0, 1.0]])
    hu = K @ (R @ e1 * sc[0])
    hv = K @ (R @ e2 * sc[1])
    hc = K @ (R @ mean + t[:, None])
    H = np.stack([hu, hv, hc], axis=1)          # [3 rows, 3 cols, n]
    tx, ty = tiles % tiles_x, tiles // tiles_x
    ox, oy = np.meshgrid(np.arange(tile_w), np.arange(tile_h))
    col = tx[:, None] * tile_w + ox.reshape(-1)[None]
    row = ty[:, None] * tile_h + oy.reshape(-1)[None]
    on = (col < width) & (row < height)
    px, py = col + 0.5, row + 0.5
    a = H[0][:, :, None] - px[None] * H[2][:, :, None]      # [3, n, P]
    b = H[1][:, :, None] - py[None] * H[2][:, :, None]
    wv = np.cross(a, b, axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        r2 = (wv[0] ** 2 + wv[1] ** 2) / wv[2] ** 2
    r2 = np.where(on & (wv[2] != 0) & np.isfinite(r2), r2, np.inf)
    re2 = np.minimum(rho_max * rho_max, 2.0 * np.log(sig / alpha_min))
    return r2.min(axis=1) / re2


def assert_pairs_match(b, t, s, ts, te, sm, intr, viewmat, width, height, tile, max_check=20000, seed=0):
    """The GPU pair list of one view against the oracle's (bin_view): it is
    the oracle's list, in the same order, less pairs whose tile no pixel of
    the surfel's support reaches (checked on up to max_check of them), and
    the tile ranges count the kept pairs."""
    n = 1 << 32
    ko = b["pair_tile"].astype(np.int64) * n + b["pair_surf"].astype(np.int64)
    kg = np.asarray(t, np.int64) * n + np.asarray(s, np.int64)
    keep = np.isin(ko, kg)
    assert np.array_equal(ko[keep], kg), "GPU pairs are not an ordered sub-list of the oracle's"
    drop = np.nonzero(~keep)[0]
    if drop.size > max_check:
        drop = np.random.default_rng(seed).choice(drop, max_check, replace=False)
    if drop.size:
        tiles_x = b["tiles"][0]
        m = _support_min_margin(sm, intr, viewmat, b["pair_surf"][drop].astype(np.int64),
                                b["pair_tile"][drop].astype(np.int64), tiles_x, tile[0], tile[1],
                                width, height)
        assert (m > 1.0).all(), f"{int((m <= 1.0).sum())} dropped pairs reach a covered pixel"
    cnt = np.bincount(b["pair_tile"][keep].astype(np.int64), minlength=len(ts))
    assert np.array_equal((np.asarray(te) - np.asarray(ts)).astype(np.int64), cnt[:len(ts)])
    return float(keep.mean()) if keep.size else 1.0
