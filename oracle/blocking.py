"""Blocking (reblocking) analysis of a serially correlated series, FP64 (test infrastructure
only: imported by tests, the repository smoke check and the benchmark's CPU-baseline leg,
never by the GPU library; it shares no code with it).

The paper quotes energies with statistical error bars over blocks of the random walk
(results sections); block energies are serially correlated, so their standard error comes
from a blocking analysis: at level 0 the series itself, at level l + 1 the means of
neighbouring pairs of level l (an odd last element is dropped).  At every level the
standard error of the mean is sqrt(s^2 / n) with s^2 the sample variance (n - 1
denominator), and its own uncertainty is that error / sqrt(2 (n - 1)).  The level used is
the first whose block size B = 2^l satisfies B^3 > 2 N (err_l / err_0)^4 (N the length of
the series), the criterion of Lee, Needs and Towler (Phys. Rev. E 83, 066706 (2011)); when
no level satisfies it, none is chosen (-1).

Pinned by tests/test_oracle_pins.py: a worked example by hand, the known standard error of
the mean of iid and of AR(1) series (closed forms), and invariance under shifts and
scaling of the series.
"""

from __future__ import annotations

import numpy as np


def reblock(x):
    """Levels of the blocking analysis: a list of (n, mean, err, err_err) for levels
    0, 1, ... while at least two blocks remain."""
    x = np.asarray(x, dtype=np.float64)
    out = []
    while x.shape[0] >= 2:
        n = x.shape[0]
        mean = x.sum() / n
        var = ((x - mean) ** 2).sum() / (n - 1)
        err = np.sqrt(var / n)
        out.append((n, mean, err, err / np.sqrt(2.0 * (n - 1))))
        h = n // 2
        x = 0.5 * (x[0:2 * h:2] + x[1:2 * h:2])
    return out


def optimal_level(levels):
    """First level l with (2^l)^3 > 2 N (err_l / err_0)^4, else -1."""
    if not levels:
        return -1
    N, err0 = levels[0][0], levels[0][2]
    for lvl, (_, _, err, _) in enumerate(levels):
        B = 2.0 ** lvl
        ratio = (err / err0) ** 4 if err0 > 0 else 1.0
        if B ** 3 > 2.0 * N * ratio:
            return lvl
    return -1
