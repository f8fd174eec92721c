"""Regression pin: the oracle reproduces its stored 2x2x2 results (tests/golden/c0_oracle.json).

The stored values were written by tests/golden/make_golden.py, which calls only
the oracle; they guard against silent drift of the oracle's arithmetic.
"""

import json
import os

import numpy as np

from tests.golden.make_golden import compute

HERE = os.path.dirname(os.path.abspath(__file__))


def _c(a):
    a = np.asarray(a)
    return a[..., 0] + 1j * a[..., 1]


def test_oracle_matches_stored_c0_results():
    with open(os.path.join(HERE, "golden", "c0_oracle.json")) as f:
        ref = json.load(f)
    now = compute()
    for key in ("energy_initial", "energy_after_step", "logdet_after_step"):
        np.testing.assert_allclose(_c(now[key]), _c(ref[key]), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(now["weight_after_step"], ref["weight_after_step"], rtol=1e-12)
