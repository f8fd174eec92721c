"""GPU parity of the comb population control against the oracle (bit-exact: the parents
are integer results of FP64 comparisons made in the same order on both sides, and the
walker state is copied, not computed).  Marked gpu: run on an MI355X."""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from oracle import walkers as wk
    from tests.gpu_cases import build, host


def _weights(rng, W, nzero):
    w = rng.exponential(size=W)
    if nzero:
        w[rng.choice(W, nzero, replace=False)] = 0.0
    return w


def _check(p, w, xi, status0=None):
    U0, G0, ld0 = host(p.U).copy(), host(p.Gh).copy(), host(p.logdet).copy()
    st0 = (np.arange(p.nwalk, dtype=np.int32) * 3 % 7) if status0 is None else status0
    p.status.copy_(torch.from_numpy(st0))
    p.weight.copy_(torch.from_numpy(w))
    par = p.population_control(xi)
    torch.cuda.synchronize()
    U1, G1, ld1, st1, w1, par_ref = wk.population_control(U0, G0, ld0, st0, w, xi)
    assert np.array_equal(host(par), par_ref)
    assert np.array_equal(host(p.U), U1)
    assert np.array_equal(host(p.Gh), G1)
    assert np.array_equal(host(p.logdet), ld1)
    assert np.array_equal(host(p.status), st1)
    assert np.array_equal(host(p.weight), w1)
    return par_ref


@pytest.mark.parametrize("case,nzero,xi", [
    ("c0", 1, 0.25), ("wide", 7, 0.0), ("wide", 0, 0.999999), ("line3", 3, 0.5)])
def test_population_control_matches_oracle(case, nzero, xi):
    s, U, x, p, pre = build(case)
    rng = np.random.default_rng(11)
    _check(p, _weights(rng, p.nwalk, nzero), xi)


def test_population_control_many_walkers():
    # more walkers than one workgroup has threads: strided comb and copy loops
    s, U, x, p, pre = build(((2, 1, 1), 6, 2, 9, 300, "random", "dense"))
    rng = np.random.default_rng(5)
    par = _check(p, _weights(rng, 300, 60), 0.37)
    assert len(set(par.tolist())) < 300


def test_population_control_degenerate_weights():
    s, U, x, p, pre = build("aniso")
    W = p.nwalk
    # all dead: unchanged, identity parents
    par = _check(p, np.zeros(W), 0.5)
    assert par.tolist() == list(range(W))
    # one survivor takes every copy
    w = np.zeros(W)
    w[2] = 0.75
    assert _check(p, w, 0.9).tolist() == [2] * W
    # equal weights: identity
    assert _check(p, np.full(W, 1.5), 0.1).tolist() == list(range(W))
    # a negative weight leaves the population unchanged
    w = np.ones(W)
    w[0] = -1.0
    assert _check(p, w, 0.2).tolist() == list(range(W))


def test_population_control_batch():
    from paper_2003_09468_amd import KptBatch
    sys_ = [build("c0")[3], build("wide")[3], build("line3")[3]]
    rng = np.random.default_rng(9)
    ws = [_weights(rng, p.nwalk, 1) for p in sys_]
    xis = [0.1, 0.6, 0.95]
    before = []
    for p, w in zip(sys_, ws):
        p.weight.copy_(torch.from_numpy(w))
        p.status.zero_()
        before.append((host(p.U).copy(), host(p.Gh).copy(), host(p.logdet).copy(),
                       host(p.status).copy()))
    b = KptBatch(sys_)
    pars = b.population_control(xis)
    torch.cuda.synchronize()
    for p, w, xi, (U0, G0, ld0, st0), par in zip(sys_, ws, xis, before, pars):
        U1, G1, ld1, st1, w1, par_ref = wk.population_control(U0, G0, ld0, st0, w, xi)
        assert np.array_equal(host(par), par_ref)
        assert np.array_equal(host(p.U), U1) and np.array_equal(host(p.Gh), G1)
        assert np.array_equal(host(p.logdet), ld1) and np.array_equal(host(p.weight), w1)
