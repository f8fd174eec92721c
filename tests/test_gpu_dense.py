"""The standard (dense) representation on the GPU: the converted system against the oracle's
conversion, and the dense system against the k-point system on the same walkers (local
energy, force-bias traces through the Coulomb energy, and one step with the mapped fields),
all through the library's kernels."""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_2003_09468_amd as lib
    from oracle import dense as dn
    from oracle import kpoint as kp
    from tests.gpu_cases import build, host, rel, phase_err

# k-point systems whose supercell fits the kernels' dense limits (nk m <= 64, nk nocc <= 16);
# self-paired Q only (c0), pairs (line3), both (mixed), Nk = 1 (mol), a larger band count
CASESEL = (["c0", "line3", "mixed", "mol", ((2, 1, 1), 20, 4, 30, 5, "random", "dense")]
           if gpu_available() else [])


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("case", CASESEL)
def test_dense_system_against_oracle(case):
    s, U, x, p, pre = build(case)
    d = p.dense(torch.from_numpy(s.H1))
    torch.cuda.synchronize()
    Ld = dn.dense_cholesky(s.L, s.mesh)
    H1d, Ad = dn.dense_one_body(s.H1, s.A)
    assert np.abs(host(d.L) - Ld).max() < 1e-15
    assert np.array_equal(host(d.A), Ad)
    xd = host(p.dense_fields(torch.from_numpy(x[0])))
    assert np.abs(xd - dn.dense_fields(x[0], s.mesh)).max() < 1e-15
    # the prepared dense system (Lh, h1h, bhalf) against the oracle's preparation of it
    pred = kp.prepare(Ld, H1d, Ad, s.dt)
    assert rel(host(d.Lh), pred["Lh"]) < 1e-13
    assert rel(host(d.bhalf), pred["bhalf"]) < 1e-13


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("case", CASESEL)
def test_dense_equals_kpoint_on_the_gpu(case):
    """Same walkers: equal local energies (total and one-body), equal Green's functions; one
    step with the mapped fields: equal walkers, log overlaps and weights."""
    s, U, x, p, pre = build(case)
    d = p.dense(torch.from_numpy(s.H1))
    d.greens()
    torch.cuda.synchronize()
    assert rel(host(d.Gh), host(p.Gh)) < 1e-12
    E, Ed = host(p.energy()), host(d.energy())
    scale = np.abs(E).sum(1).max()
    assert np.abs(E.sum(1) - Ed.sum(1)).max() < 1e-11 * scale
    assert np.abs(E[:, 0] - Ed[:, 0]).max() < 1e-12 * scale
    xt = torch.from_numpy(x[0])
    xd = p.dense_fields(xt)
    p.step(xt)
    d.step(xd)
    torch.cuda.synchronize()
    assert rel(host(d.U), host(p.U)) < 1e-11
    assert phase_err(host(d.logdet), host(p.logdet)) < 1e-11
    np.testing.assert_allclose(host(d.weight), host(p.weight), rtol=1e-10)
