"""Regression check of the oracle against its stored 64x48 summary
(written by tests/golden/make_golden.py, which calls only the oracle)."""
import json
import os

import numpy as np

from tests.golden.make_golden import summary

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_matches_stored_summary(orc):
    with open(os.path.join(HERE, "golden", "config0_oracle_summary.json")) as f:
        ref = json.load(f)
    cur = summary()
    for k, v in ref.items():
        if isinstance(v, dict):
            for kk in v:
                np.testing.assert_allclose(cur[k][kk], v[kk], rtol=1e-10, err_msg=f"{k}.{kk}")
        elif isinstance(v, str):
            assert cur[k] == v
        else:
            np.testing.assert_allclose(cur[k], v, rtol=1e-10, err_msg=k)
