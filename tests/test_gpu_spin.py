"""Two-determinant (collinear) walkers on the GPU against the oracle's spin-resolved
formulas: force bias, local energy, its adjoint, a step (walkers, log overlaps, weights),
population control and a captured block; and equal spins against the closed shell."""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_2003_09468_amd as lib
    from synth import make_system, make_walkers, make_fields, make_spin_trial, spin_view
    from oracle import kpoint as kp
    from oracle import spin as sp
    from tests.gpu_cases import host, rel, phase_err

# (mesh, m, n_up, n_dn, nchol, nwalk): different electron counts per spin, self-paired and
# paired Q, a ragged band count, nocc past 8 in one half
SPIN_CASES = {
    "c0": ((2, 2, 2), 8, 2, 1, 24, 4),
    "line3": ((3, 1, 1), 9, 4, 3, 20, 5),
    "mixed": ((1, 2, 3), 6, 2, 2, 17, 3),
    "mol": ((1, 1, 1), 11, 3, 5, 13, 4),
    "wide": ((2, 2, 1), 26, 4, 3, 40, 9),
    "occ10": ((2, 1, 1), 14, 10, 7, 19, 3),
}
CASESEL = list(SPIN_CASES) if gpu_available() else []


def build_pair(case, prec=0, seed=3):
    mesh, m, nu, nd, C, W = SPIN_CASES[case]
    s, rng = make_system(mesh, m, nu, C, seed=seed, trial="random")
    A_dn = make_spin_trial(s, nd, rng)
    U = (make_walkers(s, W, rng, kind="dense"),
         make_walkers(spin_view(s, A_dn), W, rng, kind="dense"))
    x = make_fields(s, W, 2, rng)
    pr = lib.KptSpinPair(s.mesh, m, nu, nd, C, W, s.dt, torch.from_numpy(s.L),
                         torch.from_numpy(s.A), torch.from_numpy(A_dn), prec=prec)
    pr.prepare(torch.from_numpy(s.H1))
    pr.set_walkers(torch.from_numpy(U[0]), torch.from_numpy(U[1]))
    pr.greens()
    torch.cuda.synchronize()
    pre = sp.prepare(s.L, s.H1, s.A, A_dn, s.dt)
    return s, (s.A, A_dn), U, x, pr, pre


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("case", CASESEL)
def test_spin_force_bias_energy_adjoint(case):
    s, A, U, x, pr, pre = build_pair(case)
    Gh = (host(pr.up.Gh).copy(), host(pr.dn.Gh).copy())
    for q in range(2):
        Gr, ld = kp.greens(U[q], A[q])
        assert rel(Gh[q], Gr) < 1e-12
        assert phase_err(host([pr.up, pr.dn][q].logdet), ld) < 1e-12
    pr.vbias()
    pr.local_energy()
    rng = np.random.default_rng(5)
    W = U[0].shape[0]
    gE = rng.standard_normal(W) + 1j * rng.standard_normal(W)
    g = pr.energy_backward([torch.from_numpy(gE), None])
    torch.cuda.synchronize()
    xb, X = sp.force_bias(pre["Lh"], Gh, s.mesh, s.dt)
    E = sp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    D = sp.energy_gradient(pre["Lh"], pre["h1h"], Gh, s.mesh)
    for i in range(2):  # both halves' slots hold the pair's values
        assert rel(host(pr.xbar(i)), xb) < 1e-12
        assert rel(host(pr.X(i)), X) < 1e-12
        Eg = host(pr.energy(i))
        assert np.abs(Eg - E).max() < 1e-11 * np.abs(E).sum(axis=1).max(), (i, Eg, E)
        assert rel(host(g[i]), gE[:, None, None] * D[i]) < 1e-11


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("case", ["c0", "line3", "wide", "occ10"] if gpu_available() else [])
def test_spin_step_against_oracle(case):
    s, A, U, x, pr, pre = build_pair(case)
    W = U[0].shape[0]
    w0 = np.linspace(0.5, 1.5, W)
    for h in (pr.up, pr.dn):
        h.weight.copy_(torch.from_numpy(w0))
        h.set_etrial(-0.7)
    ld = tuple(kp.greens(U[q], A[q])[1] for q in range(2))
    pr.step(pr.step_fields(torch.from_numpy(x[:1])), ortho=False, energy=True)
    torch.cuda.synchronize()
    r = sp.step(U, ld, w0, x[0], pre, A, s.L, s.mesh, s.dt, etrial=-0.7)
    for q, h in enumerate((pr.up, pr.dn)):
        assert rel(host(h.U), r["U"][q]) < 1e-11
        assert phase_err(host(h.logdet), r["logdet"][q]) < 1e-11
        np.testing.assert_allclose(host(h.weight), r["weight"], rtol=1e-10, atol=1e-300)
    assert torch.equal(pr.up.weight, pr.dn.weight)
    assert torch.equal(pr.up.status, pr.dn.status)
    E = sp.local_energy(pre["Lh"], pre["h1h"], r["Gh"], s.mesh)
    for i in range(2):
        Eg = host(pr.energy(i))
        assert np.abs(Eg - E).max() < 1e-10 * np.abs(E).sum(axis=1).max()


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("prec", [0, 2] if gpu_available() else [])
def test_equal_spins_equal_closed_shell(prec):
    """Equal up and down halves reproduce the closed-shell problem: force bias, walkers,
    log overlaps and weights bit for bit (the halves' means of equal values), the energy to
    rounding (its Coulomb sum runs in another order)."""
    from tests.gpu_cases import build
    s, U, x, p, pre = build("wide", prec=prec)
    pr = lib.KptSpinPair(s.mesh, s.m, s.nocc, s.nocc, s.nchol, U.shape[0], s.dt,
                         torch.from_numpy(s.L), torch.from_numpy(s.A), torch.from_numpy(s.A),
                         prec=prec)
    pr.prepare(torch.from_numpy(s.H1))
    pr.set_walkers(torch.from_numpy(U), torch.from_numpy(U))
    pr.greens()
    cb = lib.KptBatch([p])
    pr.step(pr.step_fields(torch.from_numpy(x)), ortho=True, energy=True)
    cb.step(cb.fields([torch.from_numpy(x)]), ortho=True, energy=True)
    torch.cuda.synchronize()
    for h in (pr.up, pr.dn):
        assert torch.equal(h.U, p.U) and torch.equal(h.Gh, p.Gh)
        assert torch.equal(h.logdet, p.logdet) and torch.equal(h.weight, p.weight)
    assert torch.equal(pr.xbar(0), cb.xbar(0)) and torch.equal(pr.xbar(1), cb.xbar(0))
    E, Ec = host(pr.energy(0)), host(cb.energy(0))
    assert np.array_equal(E[:, [0, 2]], Ec[:, [0, 2]])
    assert np.abs(E[:, 1] - Ec[:, 1]).max() < 1e-13 * np.abs(Ec[:, 1]).max()


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_spin_population_and_graph():
    """The comb gives both halves the same copies; a captured block over a batch of a
    closed-shell system and a pair equals the eager step of an identical batch."""
    from tests.gpu_cases import build
    s, A, U, x, pr, pre = build_pair("wide")
    W = U[0].shape[0]
    for h in (pr.up, pr.dn):
        h.weight.copy_(torch.linspace(0.1, 2.0, W, dtype=torch.float64))
    par = pr.population_control([0.37, 0.91])  # the down half's xi is not read
    torch.cuda.synchronize()
    assert torch.equal(par[0], par[1])
    assert torch.equal(pr.up.weight, pr.dn.weight)
    idx = host(par[0])
    assert np.array_equal(host(pr.up.U), U[0][idx])
    assert np.array_equal(host(pr.dn.U), U[1][idx])

    def make():
        _, _, xc, pc, _ = build("c0")
        _, _, _, x2, p2, _ = build_pair("wide")
        b = lib.KptBatch([pc, p2.up, p2.dn])
        return b, b.fields([torch.from_numpy(v) for v in (xc, x2, x2)]), (pc, p2.up, p2.dn)

    b1, f1, h1 = make()
    b2, f2, h2 = make()
    b1.step(f1, ortho=True, energy=True)
    g = b2.graph(f2, ortho=True, energy=True)
    g.launch()
    torch.cuda.synchronize()
    for a, b in zip(h1, h2):
        assert torch.equal(a.U, b.U) and torch.equal(a.weight, b.weight)
        assert torch.equal(a.logdet, b.logdet) and torch.equal(a.Gh, b.Gh)
    for i in range(3):
        assert torch.equal(b1.energy(i), b2.energy(i))
    g.close()


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_equal_spins_placed_int8_energy():
    """Equal halves in the placed BF16X3-step / INT8X5-energy precision reproduce the
    closed shell in the same placement: steps bit for bit, one-body and exchange energies
    bit for bit (the halves' means of equal values), the Coulomb energy to rounding."""
    from tests.gpu_cases import build
    pl = lib.prec_place(lib.PREC_BF16X3, lib.PREC_INT8X5)
    s, U, x, p, pre = build("wide", prec=pl)
    pr = lib.KptSpinPair(s.mesh, s.m, s.nocc, s.nocc, s.nchol, U.shape[0], s.dt,
                         torch.from_numpy(s.L), torch.from_numpy(s.A), torch.from_numpy(s.A),
                         prec=pl)
    pr.prepare(torch.from_numpy(s.H1))
    pr.set_walkers(torch.from_numpy(U), torch.from_numpy(U))
    pr.greens()
    cb = lib.KptBatch([p])
    pr.step(pr.step_fields(torch.from_numpy(x)), ortho=True, energy=True)
    cb.step(cb.fields([torch.from_numpy(x)]), ortho=True, energy=True)
    torch.cuda.synchronize()
    for h in (pr.up, pr.dn):
        assert torch.equal(h.U, p.U) and torch.equal(h.weight, p.weight)
    E, Ec = host(pr.energy(0)), host(cb.energy(0))
    assert np.array_equal(E[:, [0, 2]], Ec[:, [0, 2]])
    assert np.abs(E[:, 1] - Ec[:, 1]).max() < 1e-13 * np.abs(Ec[:, 1]).max()
    assert np.array_equal(host(pr.energy(1)), E)


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
def test_spin_energy_noalloc_equals_energy():
    """The entry point without a workspace gives a pair the same energies, bit for bit."""
    import ctypes
    from paper_2003_09468_amd import binding as Bd
    s, A, U, x, pr, pre = build_pair("line3")
    pr.local_energy()
    torch.cuda.synchronize()
    E = [host(pr.energy(i)).copy() for i in range(2)]
    out = torch.zeros_like(pr._E)
    Bd.check("afqmc_kpt_energy_noalloc",
             Bd.lib().afqmc_kpt_energy_noalloc(pr.arr, 2, out.data_ptr(), Bd._stream()))
    torch.cuda.synchronize()
    for i in range(2):
        got = host(pr._view(out, "energy", i, torch.complex128, (pr.problems[i].nwalk, 3)))
        assert np.array_equal(got, E[i])
