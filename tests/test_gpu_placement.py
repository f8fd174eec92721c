"""Precision placement: BF16X3 step contractions with an FP64 local energy and adjoint
(and the reverse), against the single-precision problems and the FP64 oracle.

A placed problem runs each stage with the kernels of that stage's precision, so its step is
bit-identical to the BF16X3 problem's and its energy and adjoint to the FP64 problem's on
the same Green's function; the energy also meets the FP64 oracle bar.
"""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_2003_09468_amd as lib
    from oracle import kpoint as kp
    from tests.gpu_cases import CASES, build, host, rel, energy_err, overlap_cond

CASESEL = ["c0", "wide", "m40", "occ10"] if gpu_available() else []


@pytest.mark.parametrize("case", CASESEL)
def test_bf16x3_step_fp64_energy(case):
    pl = lib.prec_place(lib.PREC_BF16X3, lib.PREC_FP64)
    s, U, x, p, pre = build(case, prec=pl)
    _, _, _, pb, _ = build(case, prec=lib.PREC_BF16X3)
    _, _, _, pd, _ = build(case, prec=lib.PREC_FP64)
    assert p.Ls is not None and p.Lhs is not None and p.L32 is None
    # energy and adjoint on the initial Gh: the FP64 kernels, bit for bit, and the oracle
    E, Ed = host(p.energy()), host(pd.energy())
    assert np.array_equal(E, Ed)
    Gh, ld = kp.greens(U, s.A)
    Eref = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    assert energy_err(E, Eref, s.nk, overlap_cond(U, s.A)) <= 1.0
    D, Dd = host(p.energy_backward()), host(pd.energy_backward())
    assert np.array_equal(D, Dd)
    assert rel(D, kp.energy_gradient(pre["Lh"], pre["h1h"], Gh, s.mesh)) < 1e-10
    # one step: the BF16X3 kernels, bit for bit
    xt = torch.from_numpy(x[0])
    _, v = p.step(xt)
    _, vb = pb.step(xt)
    torch.cuda.synchronize()
    assert v.dtype == torch.complex64
    assert torch.equal(v, vb)
    assert torch.equal(p.U, pb.U) and torch.equal(p.Gh, pb.Gh)
    assert torch.equal(p.weight, pb.weight)
    out = kp.step(U, ld, np.ones(U.shape[0]), x[0], pre, s.A, s.L, s.mesh, s.dt)
    assert rel(host(p.U), out["U"]) < 5e-5
    # the energy after the step: FP64 kernels on the BF16X3-propagated Gh
    pd.Gh.copy_(p.Gh)
    assert np.array_equal(host(p.energy()), host(pd.energy()))


@pytest.mark.parametrize("case", ["c0", "wide"] if gpu_available() else [])
def test_fp64_step_bf16x3_energy(case):
    pl = lib.prec_place(lib.PREC_FP64, lib.PREC_BF16X3)
    s, U, x, p, pre = build(case, prec=pl)
    _, _, _, pb, _ = build(case, prec=lib.PREC_BF16X3)
    _, _, _, pd, _ = build(case, prec=lib.PREC_FP64)
    assert p.Ls is None and p.Lhs is not None
    assert np.array_equal(host(p.energy()), host(pb.energy()))
    assert np.array_equal(host(p.energy_backward()), host(pb.energy_backward()))
    xt = torch.from_numpy(x[0])
    _, v = p.step(xt)
    _, vd = pd.step(xt)
    torch.cuda.synchronize()
    assert v.dtype == torch.complex128 and torch.equal(v, vd)
    assert torch.equal(p.U, pd.U) and torch.equal(p.weight, pd.weight)


@pytest.mark.parametrize("case", ["wide"] if gpu_available() else [])
def test_placed_step_block_energy(case):
    """afqmc_kpt_step with the energy flag evaluates the final energy in the energy
    precision: the placed block's energy equals the FP64 energy of its own final Gh."""
    pl = lib.prec_place(lib.PREC_BF16X3, lib.PREC_FP64)
    s, U, x, p, pre = build(case, prec=pl)
    _, _, _, pd, _ = build(case, prec=lib.PREC_FP64)
    b = lib.KptBatch([p])
    f = b.fields([torch.from_numpy(x)])
    b.step(f, ortho=True, energy=True)
    E = host(b.energy(0)).copy()
    pd.Gh.copy_(p.Gh)
    assert np.array_equal(E, host(pd.energy()))


@pytest.mark.parametrize("case", ["wide", "m40"] if gpu_available() else [])
def test_reduced_green_function_product(case):
    """AFQMC_PROPAGATE_REDUCED_GH: in a reduced step precision the new Gh comes from the FP32
    product; the walkers, log overlaps, weights and status are those of the FP64 product bit
    for bit, Gh agrees to FP32 rounding; FP64 problems ignore the flag; afqmc_kpt_step uses it
    for every step whose Gh only feeds the next force bias."""
    for prec in (lib.PREC_BF16X3, lib.PREC_FP32, lib.PREC_FP64):
        s, U, x, p, pre = build(case, prec=prec)
        _, _, _, q, _ = build(case, prec=prec)
        xt = torch.from_numpy(x[0])
        p.step(xt, reduced_gh=True)
        q.step(xt)
        torch.cuda.synchronize()
        for k in ("U", "logdet", "weight", "status"):
            assert torch.equal(getattr(p, k), getattr(q, k)), (prec, k)
        if prec == lib.PREC_FP64:
            assert torch.equal(p.Gh, q.Gh)
        else:
            assert rel(host(p.Gh), host(q.Gh)) < 2e-6
    # the block entry: reduced Gh for the first step, FP64 after the re-orthonormalisation
    s, U, x, p, pre = build(case, prec=lib.PREC_BF16X3)
    _, _, _, q, _ = build(case, prec=lib.PREC_BF16X3)
    b = lib.KptBatch([p])
    b.step(b.fields([torch.from_numpy(x)]), ortho=True, energy=False)
    for it in range(x.shape[0]):
        q.step(torch.from_numpy(x[it]), ortho=(it == x.shape[0] - 1), reduced_gh=True)
    torch.cuda.synchronize()
    for k in ("U", "Gh", "logdet", "weight", "status"):
        assert torch.equal(getattr(p, k), getattr(q, k)), k
