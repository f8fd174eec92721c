"""The reduced-precision contraction modes against the FP64 oracle, on the six parity cases.

FP32 (complex64 operands, FP32 MFMA accumulation): a K-term dot product carries a
relative error of about sqrt(K) * 2^-24 of sum |a b| (inputs rounded once from FP64, K up
to a few hundred here), i.e. ~1e-6; the bars are 5e-6 relative to the largest reference
entry for the force bias, HS potential and propagated walkers, 2e-5 for the energy adjoint
(two chained contractions), and 5e-6 of the summed magnitude of the three energy parts per
walker for E_L (the parts cancel, so their size, not |E|, sets the rounding scale).

BF16X3 (force bias, HS potential, Taylor terms and exchange on the three-pass BF16 split,
the rest FP32): each split operand keeps 16 significant bits plus a rounded remainder and
the lo*lo term is dropped, so a product carries ~2^-16 relative error (~1.5e-5) before
FP32 accumulation; the bars are 1e-4 of the largest entry for the force bias and the HS
potential and of the largest magnitude for the exchange energy, 5e-5 of the summed part
magnitudes on E_L, and 5e-5 for one propagated step (the potential enters the propagator
multiplied by sqrt(dt)).
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from oracle import kpoint as kp
    from tests.gpu_cases import CASES, build, host, rel

ALL = list(CASES) if gpu_available() else []


@pytest.mark.parametrize("case", ALL)
@pytest.mark.parametrize("prec", [1, 2], ids=["fp32", "bf16x3"])
def test_contractions_and_step(case, prec):
    s, U, x, p, pre = build(case, prec=prec)
    Gh, ld = kp.greens(U, s.A)
    xbar, X = kp.force_bias(pre["Lh"], Gh, s.mesh, s.dt)
    xb, Xg = p.vbias()
    assert rel(host(Xg), X) < (5e-6 if prec == 1 else 1e-4)
    zeta = kp.combined_field(x[0], xbar, s.mesh)
    vref = kp.hs_potential(s.L, zeta, s.mesh)
    v = p.vhs(torch.from_numpy(x[0]), xb)
    assert rel(host(v), vref) < (5e-6 if prec == 1 else 1e-4)
    out = kp.step(U, ld, np.ones(U.shape[0]), x[0], pre, s.A, s.L, s.mesh, s.dt)
    p.propagate(v, torch.from_numpy(x[0]), xb)
    torch.cuda.synchronize()
    assert rel(host(p.U), out["U"]) < (5e-6 if prec == 1 else 5e-5)


@pytest.mark.parametrize("case", ALL)
@pytest.mark.parametrize("prec", [1, 2], ids=["fp32", "bf16x3"])
def test_energy_and_adjoint(case, prec):
    s, U, x, p, pre = build(case, prec=prec)
    Gh, _ = kp.greens(U, s.A)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    Eg = host(p.energy())
    scale = np.abs(E).sum(1)
    bar = 5e-6 if prec == 1 else 5e-5
    assert (np.abs(Eg.sum(1) - E.sum(1)) / scale).max() < bar
    if prec == 2:
        assert np.abs(Eg[:, 2] - E[:, 2]).max() / np.abs(E[:, 2]).max() < 1e-4
    D = kp.energy_gradient(pre["Lh"], pre["h1h"], Gh, s.mesh)
    assert rel(host(p.energy_backward()), D) < 2e-5


@pytest.mark.parametrize("shape", [((3, 3, 1), 14, 12, 12, 5, "random", "dense"),
                                   ((4, 4, 2), 6, 5, 10, 3, "random", "dense")],
                         ids=["n108", "n160"])
def test_bf16x3_step_wide_column_tiles(shape):
    """BF16X3 Taylor terms with 108 walker columns (seven 16-column blocks, the 3x3x3
    workload's width) and with 160 (two column tiles); one step against the oracle."""
    s, U, x, p, pre = build(shape, prec=2)
    Gh, ld = kp.greens(U, s.A)
    out = kp.step(U, ld, np.ones(U.shape[0]), x[0], pre, s.A, s.L, s.mesh, s.dt)
    p.step(torch.from_numpy(x[0]))
    torch.cuda.synchronize()
    assert rel(host(p.U), out["U"]) < 5e-5


@pytest.mark.parametrize("shape", [((2, 1, 1), 40, 4, 30, 21, "random", "dense"),
                                   ((1, 2, 1), 36, 3, 22, 9, "random", "dense")],
                         ids=["m40_nocc4", "m36_nocc3"])
def test_bf16x3_energy_two_k_blocks(shape):
    """BF16X3 exchange with m > 32 (two 32-wide K blocks per MFMA chain, one column tile
    per wave): the nocc = 4 kernel and the general one, ragged walker chunks."""
    s, U, x, p, pre = build(shape, prec=2)
    Gh, _ = kp.greens(U, s.A)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    Eg = host(p.energy())
    scale = np.abs(E).sum(1)
    assert (np.abs(Eg.sum(1) - E.sum(1)) / scale).max() < 5e-5
    assert np.abs(Eg[:, 2] - E[:, 2]).max() / np.abs(E[:, 2]).max() < 1e-4
