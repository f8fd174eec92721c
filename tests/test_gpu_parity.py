"""GPU parity: every entry point of the C ABI against the FP64 oracle, element by element.

FP64 bar: the energy within 1e-10 Ha per cell (absolute) and every other array
within 1e-11 relative to its largest entry; both sides consume the same seeded
arrays.  Marked gpu: run on an MI355X.
"""

import math

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from oracle import kpoint as kp
    from tests.gpu_cases import CASES, build, host, rel, phase_err, energy_err, overlap_cond

ALL = list(CASES) if gpu_available() else []


@pytest.mark.parametrize("case", ALL)
def test_prepare(case):
    s, U, x, p, pre = build(case)
    assert rel(host(p.Lh), pre["Lh"]) < 1e-13
    assert rel(host(p.h1h), pre["h1h"]) < 1e-13
    assert rel(host(p.bhalf), pre["bhalf"]) < 1e-13


@pytest.mark.parametrize("case", ALL)
def test_greens(case):
    s, U, x, p, pre = build(case)
    Gh, ld = kp.greens(U, s.A)
    assert rel(host(p.Gh), Gh) < 1e-11
    assert phase_err(host(p.logdet), ld) < 1e-11
    assert np.all(np.abs(host(p.logdet).imag) <= math.pi + 1e-12)
    assert int(host(p.status).max()) == 0


@pytest.mark.parametrize("case", ALL)
def test_vbias(case):
    s, U, x, p, pre = build(case)
    Gh, _ = kp.greens(U, s.A)
    xbar, X = kp.force_bias(pre["Lh"], Gh, s.mesh, s.dt)
    xb, Xg = p.vbias()
    assert rel(host(Xg), X) < 1e-11
    assert rel(host(xb), xbar) < 1e-11


@pytest.mark.parametrize("case", ALL)
def test_vhs(case):
    s, U, x, p, pre = build(case)
    Gh, _ = kp.greens(U, s.A)
    xbar, _ = kp.force_bias(pre["Lh"], Gh, s.mesh, s.dt)
    zeta = kp.combined_field(x[0], xbar, s.mesh)
    vref = kp.hs_potential(s.L, zeta, s.mesh)
    xb, _ = p.vbias()
    v = p.vhs(torch.from_numpy(x[0]), xb)
    assert rel(host(v), vref) < 1e-11


@pytest.mark.parametrize("case", ALL)
def test_propagate_and_weights(case):
    s, U, x, p, pre = build(case)
    Gh, ld = kp.greens(U, s.A)
    out = kp.step(U, ld, np.ones(U.shape[0]), x[0], pre, s.A, s.L, s.mesh, s.dt)
    p.step(torch.from_numpy(x[0]))
    torch.cuda.synchronize()
    assert rel(host(p.U), out["U"]) < 1e-11
    assert rel(host(p.Gh), out["Gh"]) < 1e-10
    assert phase_err(host(p.logdet), out["logdet"]) < 1e-10
    np.testing.assert_allclose(host(p.weight), out["weight"], rtol=1e-10, atol=1e-14)
    st = host(p.status)
    killed = out["weight"] == 0.0
    assert np.all(((st & 4) != 0) == killed)


@pytest.mark.parametrize("case", ALL)
def test_orthonormalize(case):
    s, U, x, p, pre = build(case)
    Ub = U * 2.0 + 0.3 * np.roll(U, 1, axis=2)
    p.set_walkers(torch.from_numpy(Ub))
    p.orthonormalize()
    torch.cuda.synchronize()
    Q = kp.orthonormalize(Ub)
    Gh, ld = kp.greens(Q, s.A)
    assert rel(host(p.U), Q) < 1e-11
    assert rel(host(p.Gh), Gh) < 1e-10
    assert phase_err(host(p.logdet), ld) < 1e-10


@pytest.mark.parametrize("case", ALL)
def test_energy(case):
    s, U, x, p, pre = build(case)
    Gh, _ = kp.greens(U, s.A)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    Eg = host(p.energy())
    # every part: 1e-10 Ha per cell, or the FP64 floor 2 eps cond(O) |parts| where larger
    assert energy_err(Eg, E, s.nk, overlap_cond(U, s.A)) <= 1.0


@pytest.mark.parametrize("case", ALL)
def test_energy_at_trial_is_real_hf(case):
    from oracle import supercell as sc
    s, U, x, p, pre = build(case)
    Af = sc.block_diag(s.A)
    p.set_walkers(torch.from_numpy(np.repeat(Af[None], U.shape[0], axis=0)))
    p.greens()
    Eg = host(p.energy())
    Gh, _ = kp.greens(Af[None], s.A)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)[0]
    assert energy_err(Eg, np.broadcast_to(E[None], Eg.shape), s.nk, np.ones(len(Eg))) <= 1.0
    assert np.abs(Eg.imag).max() < 1e-10


@pytest.mark.parametrize("case", ALL)
def test_energy_backward(case):
    s, U, x, p, pre = build(case)
    Gh, _ = kp.greens(U, s.A)
    D = kp.energy_gradient(pre["Lh"], pre["h1h"], Gh, s.mesh)
    g = host(p.energy_backward())
    assert rel(g, D) < 1e-11
    rng = np.random.default_rng(1)
    gE = rng.standard_normal(U.shape[0]) + 1j * rng.standard_normal(U.shape[0])
    g2 = host(p.energy_backward(gE=torch.from_numpy(gE).cuda()))
    assert rel(g2, gE[:, None, None] * D) < 1e-11


def test_autograd_convention():
    from paper_2003_09468_amd import local_energy
    s, U, x, p, pre = build("aniso")
    Gh, _ = kp.greens(U, s.A)
    D = kp.energy_gradient(pre["Lh"], pre["h1h"], Gh, s.mesh)
    G = p.Gh.clone().requires_grad_(True)
    E = local_energy(p, G)
    rng = np.random.default_rng(2)
    c = torch.from_numpy(rng.standard_normal(U.shape[0]) + 1j * rng.standard_normal(U.shape[0])).cuda()
    # real loss L = Re(sum c E): dL/dconj(G) convention gives grad = conj(c) ... torch: grad = c* dE/dG *
    loss = (c * E).real.sum()
    loss.backward()
    expect = np.conj(host(c)[:, None, None] * D)
    assert rel(host(G.grad), expect) < 1e-11
    Eref = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh).sum(1)
    assert energy_err(host(E)[:, None], Eref[:, None], s.nk, overlap_cond(U, s.A)) <= 1.0


def test_two_steps_then_energy_c0():
    """Trajectory parity: two propagation steps (the second with re-orthonormalisation) + energy."""
    s, U, x, p, pre = build("c0")
    Gh, ld = kp.greens(U, s.A)
    w = np.ones(U.shape[0])
    Ur = U
    for it in range(2):
        out = kp.step(Ur, ld, w, x[it], pre, s.A, s.L, s.mesh, s.dt)
        Ur, ld, w = out["U"], out["logdet"], out["weight"]
        p.step(torch.from_numpy(x[it]), ortho=(it == 1))
    Ur = kp.orthonormalize(Ur)
    Gh, ld = kp.greens(Ur, s.A)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    Eg = host(p.energy())
    assert energy_err(Eg, E, s.nk, overlap_cond(Ur, s.A)) <= 1.0
    np.testing.assert_allclose(host(p.weight), w, rtol=1e-10)
    assert rel(host(p.U), Ur) < 1e-10


# ---------------------------------------------------------------------------
# degenerate cases

def test_singular_walker_flagged():
    s, U, x, p, pre = build("aniso")
    Ub = U.copy()
    Ub[1][:, 0] = 0.0  # a walker orthogonal to the trial: det O = 0
    p.set_walkers(torch.from_numpy(Ub))
    p.greens()
    st = host(p.status)
    assert st[1] & 1
    assert np.all(st[[0, 2, 3, 4, 5]] == 0)
    assert np.all(np.isfinite(host(p.Gh)))
    p.step(torch.from_numpy(x[0]))
    wt = host(p.weight)
    assert wt[1] == 0.0
    # the other walkers evolve exactly as without the singular one
    keep = [0, 2, 3, 4, 5]
    Gh, ld = kp.greens(U[keep], s.A)
    out = kp.step(U[keep], ld, np.ones(len(keep)), x[0][keep], pre, s.A, s.L, s.mesh, s.dt)
    np.testing.assert_allclose(wt[keep], out["weight"], rtol=1e-10, atol=0)
    assert rel(host(p.U)[keep], out["U"]) < 1e-11


def test_nonfinite_field_flagged():
    s, U, x, p, pre = build("aniso")
    xx = x[0].copy()
    xx[2, 0, 0, 0] = np.nan
    xb, _ = p.vbias()
    v = p.vhs(torch.from_numpy(xx), xb)
    p.propagate(v, torch.from_numpy(xx), xb)
    st = host(p.status)
    assert st[2] & 2
    assert host(p.weight)[2] == 0.0


def test_phaseless_kill():
    """Forced from the host: shifting the stored log overlap's phase by 0.3 pi makes the
    overlap-ratio angle exceed pi/2 (weight -> 0, KILLED); a 0.05 pi shift does not."""
    s, U, x, p, pre = build("mol")
    Gh, ld = kp.greens(U, s.A)
    shift = np.zeros(U.shape[0])
    shift[0], shift[1] = 0.3 * math.pi, 0.05 * math.pi
    ld_old = ld + 1j * shift
    out = kp.step(U, ld_old, np.ones(U.shape[0]), x[0], pre, s.A, s.L, s.mesh, s.dt)
    p.logdet.copy_(torch.from_numpy(ld_old))
    p.step(torch.from_numpy(x[0]))
    wt, st = host(p.weight), host(p.status)
    assert wt[0] == 0.0 and (st[0] & 4)
    assert wt[1] > 0.0 and not (st[1] & 4)
    np.testing.assert_allclose(wt, out["weight"], rtol=1e-10, atol=0)


def test_determinism():
    s, U, x, p, pre = build("line3")
    E1 = host(p.energy())
    E2 = host(p.energy())
    assert np.array_equal(E1, E2)
    p.step(torch.from_numpy(x[0]))
    U1 = host(p.U)
    p.set_walkers(torch.from_numpy(U))
    p.greens()
    p.step(torch.from_numpy(x[0]))
    assert np.array_equal(U1, host(p.U))


# ---------------------------------------------------------------------------
# occupied dimension above 128: the blocked inverse and the L2-resident Cholesky

def test_large_occupied_dimension():
    """nk*nocc = 160: Green's function, log overlap, energy, one step and the QR."""
    s, U, x, p, pre = build(((4, 4, 2), 6, 5, 10, 3, "random", "dense"))
    Gh, ld = kp.greens(U, s.A)
    assert rel(host(p.Gh), Gh) < 1e-11
    assert phase_err(host(p.logdet), ld) < 1e-11
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    assert energy_err(host(p.energy()), E, s.nk, overlap_cond(U, s.A)) <= 1.0
    out = kp.step(U, ld, np.ones(U.shape[0]), x[0], pre, s.A, s.L, s.mesh, s.dt)
    p.step(torch.from_numpy(x[0]))
    assert rel(host(p.U), out["U"]) < 1e-11
    assert rel(host(p.Gh), out["Gh"]) < 1e-10
    assert phase_err(host(p.logdet), out["logdet"]) < 1e-10
    check_ortho(p, s, host(p.U))


def check_ortho(p, s, Ub):
    """Re-orthonormalise the GPU's walkers and compare with the oracle's QR of them; the
    QR adds no status bits."""
    st0 = host(p.status).copy()
    p.orthonormalize()
    torch.cuda.synchronize()
    Q = kp.orthonormalize(Ub)
    Gh, ld = kp.greens(Q, s.A)
    assert rel(host(p.U), Q) < 1e-11
    assert rel(host(p.Gh), Gh) < 1e-10
    assert phase_err(host(p.logdet), ld) < 1e-10
    assert np.array_equal(host(p.status), st0)


def test_greens_at_maximum_occupied_dimension():
    """nk*nocc = 256, the largest the inverse and the Cholesky take."""
    s, U, x, p, pre = build(((4, 4, 4), 5, 4, 4, 2, "random", "dense"))
    Gh, ld = kp.greens(U, s.A)
    assert rel(host(p.Gh), Gh) < 1e-10
    assert phase_err(host(p.logdet), ld) < 1e-10
    assert int(host(p.status).max()) == 0
    Ub = U * 2.0 + 0.3 * np.roll(U, 1, axis=2)
    p.set_walkers(torch.from_numpy(Ub))
    check_ortho(p, s, Ub)


def test_large_ortho_rank_deficient_walker():
    """nk*nocc = 160: a walker with a zero orbital has a singular overlap matrix S = U^H U;
    it is flagged and left unchanged, the others are re-orthonormalised."""
    s, U, x, p, pre = build(((4, 4, 2), 6, 5, 10, 3, "random", "dense"))
    Ub = U.copy()
    Ub[1][:, 7] = 0.0
    p.set_walkers(torch.from_numpy(Ub))
    p.orthonormalize()
    torch.cuda.synchronize()
    st = host(p.status)
    assert st[1] & 1
    assert st[0] == 0 and st[2] == 0
    Uo = host(p.U)
    assert np.array_equal(Uo[1], Ub[1])
    Q = kp.orthonormalize(Ub[[0, 2]])
    assert rel(Uo[[0, 2]], Q) < 1e-11


# ---------------------------------------------------------------------------
# occupied dimensions at the limits of the register-resident inverse (nk*nocc = 112) and of
# the LDS-resident Cholesky factor (128: every row of the four-lanes-per-row kernel in use)

@pytest.mark.parametrize("nocc", [14, 16])
def test_inverse_and_cholesky_size_limits(nocc):
    """nk*nocc = 112 and 128 on a 2x2x2 mesh: Green's function, log overlap and the QR."""
    s, U, x, p, pre = build(((2, 2, 2), 17, nocc, 9, 3, "random", "dense"))
    Gh, ld = kp.greens(U, s.A)
    assert rel(host(p.Gh), Gh) < 1e-10
    assert phase_err(host(p.logdet), ld) < 1e-10
    assert int(host(p.status).max()) == 0
    Ub = U * 2.0 + 0.3 * np.roll(U, 1, axis=2)
    p.set_walkers(torch.from_numpy(Ub))
    check_ortho(p, s, Ub)


def test_lds_ortho_rank_deficient_walker():
    """nk*nocc = 128 (the LDS Cholesky): a walker with a zero orbital is flagged and left
    unchanged, the others are re-orthonormalised."""
    s, U, x, p, pre = build(((2, 2, 2), 17, 16, 9, 3, "random", "dense"))
    Ub = U.copy()
    Ub[1][:, 11] = 0.0
    p.set_walkers(torch.from_numpy(Ub))
    p.orthonormalize()
    torch.cuda.synchronize()
    st = host(p.status)
    assert st[1] & 1
    assert st[0] == 0 and st[2] == 0
    Uo = host(p.U)
    assert np.array_equal(Uo[1], Ub[1])
    Q = kp.orthonormalize(Ub[[0, 2]])
    assert rel(Uo[[0, 2]], Q) < 1e-11


def test_mixed_energy():
    """The weighted average of the walkers' energies after a step, on the GPU's own energies
    and weights, against the oracle's formula; also on every system of a batch."""
    from paper_2003_09468_amd import KptBatch
    s, U, x, p, pre = build("line3")
    p.step(torch.from_numpy(x[0]))
    E = p.energy()
    Em = complex(host(p.mixed_energy(E)))
    ref = kp.mixed_energy(host(E), host(p.weight))
    assert abs(Em - ref) < 1e-12 * max(1.0, abs(ref))
    items = [build(c, seed=20 + i) for i, c in enumerate(["aniso", "mixed"])]
    b = KptBatch([it[3] for it in items])
    f = b.fields([torch.from_numpy(it[2][:1]) for it in items])
    b.step(f, energy=True)
    got = host(b.mixed_energy())
    for i, it in enumerate(items):
        ref = kp.mixed_energy(host(b.energy(i)), host(it[3].weight))
        assert abs(got[i] - ref) < 1e-12 * max(1.0, abs(ref))
