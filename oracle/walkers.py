"""Population control between blocks, FP64 (test infrastructure only).

Only tests, the repository smoke check and the benchmark's CPU-baseline leg may import
this module.  It shares no code with the GPU library.

The paper runs its walkers in blocks with error bars from blocking analysis, which
implies a branching or reconfiguration step between blocks that it does not describe.
This module takes the standard comb: nwalk equally spaced points, offset by one uniform
number xi in [0, 1), are laid over the cumulative weights, and every point copies the
walker whose weight interval contains it; the new walkers all carry the mean weight.
Pinned by properties that hold for any correct comb (tests/test_oracle_pins.py): the
copy counts are the floor or ceiling of nwalk w_i / sum(w), their average over xi is
exactly nwalk w_i / sum(w), equal weights give the identity, weight-0 walkers are never
chosen, and a worked example by hand.
"""

from __future__ import annotations

import numpy as np


def comb_parents(weight, xi):
    """Parent walker of each of the nwalk copies.

    c_i = w_0 + ... + w_i summed in walker order; copy j takes the walker i with
    c_{i-1} <= (j + xi) (c / nwalk) < c_i, no later than the last walker of positive
    weight.  Negative or non-finite weights, or a non-positive total, leave the
    population as it is (identity)."""
    w = np.asarray(weight, dtype=np.float64)
    W = w.shape[0]
    ident = np.arange(W)
    if np.any(~np.isfinite(w)) or np.any(w < 0):
        return ident
    c = np.cumsum(w)  # sequential, walker order
    tot = c[-1]
    if not (tot > 0 and np.isfinite(tot)):
        return ident
    z = (np.arange(W) + xi) * (tot / W)
    idx = np.searchsorted(c, z, side="right")
    last = int(np.flatnonzero(w > 0)[-1])
    return np.minimum(idx, last)


def population_control(U, Gh, logdet, status, weight, xi):
    """The resampled walker state (U, Gh, logdet, status, weight) and the parents; the
    new weights are all c / nwalk (unchanged when the population is left as it is)."""
    par = comb_parents(weight, xi)
    w = np.asarray(weight, dtype=np.float64)
    new_w = w.copy()
    if _valid(w):
        new_w[:] = np.cumsum(w)[-1] / w.shape[0]
    return U[par], Gh[par], logdet[par], status[par], new_w, par


def _valid(w):
    if np.any(~np.isfinite(w)) or np.any(w < 0):
        return False
    tot = np.cumsum(w)[-1]
    return bool(tot > 0 and np.isfinite(tot))
