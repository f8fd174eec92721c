"""The seeded input generator: streamed Cholesky blocks equal the stored ones."""

import numpy as np

from synth.kpt_inputs import make_system, make_walkers


def test_streamed_blocks_equal_stored():
    s, rng = make_system((2, 3, 1), 5, 3, 7, seed=4)
    U = make_walkers(s, 3, rng)
    got = {}
    s2, rng2 = make_system((2, 3, 1), 5, 3, 7, seed=4,
                           sink=lambda Q, k, b: got.__setitem__((Q, k), b.copy()))
    U2 = make_walkers(s2, 3, rng2)
    assert s2.L is None and len(got) == s.nk * s.nk
    for (Q, k), b in got.items():
        assert np.array_equal(b, s.L[Q, k])
    assert np.array_equal(U, U2) and np.array_equal(s.H1, s2.H1) and np.array_equal(s.A, s2.A)
