"""Writes the oracle regression fixture for the 64x48 / 2,000-surfel scene.

The paper prints no kernel-level worked example, so this fixture holds
values produced by the FP64 oracle itself (this script calls only
``oracle`` and the seeded scene generator).  It guards the oracle against
unintended changes; the oracle's correctness is pinned separately by the
closed forms, invariants and finite differences in test_oracle_pins.py.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2604_03092_amd import scenes  # noqa: E402


def summary():
    sc = scenes.config0()
    o = oracle.render_scene(sc)
    loss, g = oracle.l1_loss(sc, o)
    grads, dvm = oracle.backward_scene(sc, g)
    b = oracle.bin_view(sc.submaps[0], 64, 48, sc.intr[0], sc.viewmat[0])
    return dict(
        scene=sc.name,
        loss=loss,
        sum_rgb=[float(v) for v in o["rgb"].sum(1)],
        sum_depth=float(o["depth"].sum()),
        sum_normal=[float(v) for v in o["normal"].sum(1)],
        sum_alpha=float(o["alpha"].sum()),
        n_useful=int(o["n_useful"]),
        n_flagged=int(o["flags"].sum()),
        n_pairs_16x16=int(b["n_pairs"]),
        grad_l2={k: float(np.linalg.norm(v)) for k, v in grads[0].items()},
        grad_viewmat=[float(v) for v in dvm[0]],
    )


if __name__ == "__main__":
    with open(os.path.join(HERE, "config0_oracle_summary.json"), "w") as f:
        json.dump(summary(), f, indent=1, sort_keys=True)
