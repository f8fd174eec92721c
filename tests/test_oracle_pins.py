"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every oracle function is checked here against something other than itself:
closed forms, invariants, textbook routines, brute force on tiny meshes and
exact finite differences.  No GPU.
"""

import math

import numpy as np
import pytest
import scipy.linalg

from synth import make_system, make_walkers, make_fields
from oracle import kpoint as kp
from oracle import supercell as sc
from oracle import molecular as mol

# meshes that exercise: molecular, self-inverse Q, only Q=0 self-inverse,
# anisotropic linearisation, and mixed
MESHES = [(1, 1, 1), (1, 1, 2), (2, 2, 2), (3, 1, 1), (2, 3, 1), (1, 2, 3)]


def tiny(mesh, m=4, nocc=2, nchol=5, seed=11, trial="random", walkers="dense", nw=2):
    s, rng = make_system(mesh, m, nocc, nchol, seed=seed, trial=trial)
    U = make_walkers(s, nw, rng, kind=walkers)
    x = make_fields(s, nw, 1, rng)[0]
    return s, U, x


def supercell_objects(s):
    LL = sc.unfold_cholesky(s.L, s.mesh)
    return LL, sc.eri(LL), sc.block_diag(s.H1), sc.block_diag(s.A)


# ---------------------------------------------------------------------------
# index algebra and generator
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mesh", MESHES + [(4, 4, 4)])
def test_kpoint_tables_brute_force(mesh):
    kmq, negq = kp.kpoint_tables(mesh)
    nk = int(np.prod(mesh))
    vec = [(a, b, c) for a in range(mesh[0]) for b in range(mesh[1]) for c in range(mesh[2])]
    for Q in range(nk):
        assert vec[negq[Q]] == tuple((-vec[Q][i]) % mesh[i] for i in range(3))
        for k in range(nk):
            assert vec[kmq[Q, k]] == tuple((vec[k][i] - vec[Q][i]) % mesh[i] for i in range(3))
    assert np.all(negq[negq] == np.arange(nk))


@pytest.mark.parametrize("mesh", MESHES)
def test_generator_time_reversal_and_hermiticity(mesh):
    s, _, _ = tiny(mesh)
    kmq, negq = kp.kpoint_tables(mesh)
    for Q in range(s.nk):
        for k in range(s.nk):
            part = s.L[negq[Q], kmq[Q, k]].transpose(1, 0, 2)
            assert np.array_equal(np.conj(s.L[Q, k]), part)
    assert np.array_equal(s.H1, s.H1.conj().transpose(0, 2, 1))
    for k in range(s.nk):
        assert np.allclose(s.A[k].conj().T @ s.A[k], np.eye(s.nocc), atol=1e-13)


def test_generator_reproducible():
    a, ua, xa = tiny((2, 1, 1), seed=5)
    b, ub, xb = tiny((2, 1, 1), seed=5)
    assert np.array_equal(a.L, b.L) and np.array_equal(ua, ub) and np.array_equal(xa, xb)
    c, _, _ = tiny((2, 1, 1), seed=6)
    assert not np.array_equal(a.L, c.L)


def test_eri_hermitian_and_pair_symmetric():
    s, _, _ = tiny((2, 3, 1), m=3, nchol=4)
    _, v, _, _ = supercell_objects(s)
    # Hermiticity of H2 and exchange of the two electrons
    assert np.abs(v - v.transpose(2, 3, 0, 1).conj()).max() < 1e-14
    assert np.abs(v - v.transpose(1, 0, 3, 2)).max() < 1e-14


# ---------------------------------------------------------------------------
# P-1: trial determinant = Hartree-Fock energy
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mesh", [(1, 1, 1), (2, 2, 2), (2, 3, 1)])
@pytest.mark.parametrize("trial", ["identity", "random"])
def test_trial_energy_equals_slater_condon(mesh, trial):
    s, _, _ = tiny(mesh, m=4, nocc=2, nchol=5, trial=trial)
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    LL, v, h, Af = supercell_objects(s)
    Gh, _ = kp.greens(Af[None], s.A)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, mesh)[0]
    e1, ec, ex = sc.slater_condon_energy(h, v, Af)
    assert abs(E[0] - e1) < 1e-12 * max(1.0, abs(e1))
    assert abs(E[1] - ec) < 1e-12 * max(1.0, abs(ec))
    assert abs(E[2] - ex) < 1e-12 * max(1.0, abs(ex))
    assert abs(E.imag).max() < 1e-12
    assert E[2].real < 0.0


def test_trial_energy_closed_form_identity_trial():
    s, _, _ = tiny((2, 2, 2), m=5, nocc=2, nchol=6, trial="identity")
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    Af = sc.block_diag(s.A)
    Gh, _ = kp.greens(Af[None], s.A)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)[0]
    n = s.nocc
    e1 = 2.0 * sum(s.H1[k, a, a] for k in range(s.nk) for a in range(n))
    x0 = 2.0 * np.einsum("kaag->g", s.L[0][:, :n, :n, :])
    ec = 0.5 * np.sum(x0 * x0)
    ex = -np.sum(np.abs(s.L[:, :, :n, :n, :]) ** 2)
    np.testing.assert_allclose(E, [e1, ec, ex], rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------------------
# P-2: Green's function invariants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mesh", [(2, 1, 1), (2, 3, 1)])
def test_greens_invariants(mesh):
    s, U, _ = tiny(mesh, trial="random")
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    Af = sc.block_diag(s.A)
    Gh, logdet = kp.greens(U, s.A)
    for w in range(U.shape[0]):
        assert np.abs(Gh[w] @ Af.conj() - np.eye(Af.shape[1])).max() < 1e-12
        G = Af.conj() @ Gh[w]
        assert np.abs(G @ G - G).max() < 1e-12
        assert abs(np.trace(G) - s.nk * s.nocc) < 1e-12
        # independent determinant: product of LU pivots from scipy
        lu, piv = scipy.linalg.lu_factor(Af.conj().T @ U[w])
        sign = (-1) ** np.sum(piv != np.arange(len(piv)))
        ld = np.sum(np.log(np.diag(lu).astype(complex))) + (0 if sign > 0 else 1j * np.pi)
        assert abs(np.exp(ld - logdet[w]) - 1.0) < 1e-12
    # invariance under U -> U R
    rng = np.random.default_rng(0)
    R = rng.standard_normal((U.shape[2], U.shape[2])) + 1j * rng.standard_normal((U.shape[2],) * 2)
    Gh2, logdet2 = kp.greens(U @ R, s.A)
    assert np.abs(Gh2 - Gh).max() < 1e-11
    dl = np.linalg.slogdet(R)
    expect = logdet + dl[1] + 1j * np.angle(dl[0])
    assert np.abs(np.exp(logdet2 - expect) - 1.0).max() < 1e-11
    E1 = kp.local_energy(pre["Lh"], pre["h1h"], Gh, mesh)
    E2 = kp.local_energy(pre["Lh"], pre["h1h"], Gh2, mesh)
    assert np.abs(E1 - E2).max() < 1e-10


# ---------------------------------------------------------------------------
# P-3: force bias = derivative of the log overlap
# ---------------------------------------------------------------------------

def test_force_bias_is_log_overlap_derivative():
    mesh = (2, 3, 1)
    s, U, _ = tiny(mesh, m=3, nocc=1, nchol=3, trial="random")
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    LL, _, _, Af = supercell_objects(s)
    Gh, _ = kp.greens(U, s.A)
    _, X = kp.force_bias(pre["Lh"], Gh, mesh, s.dt)
    eps = 1e-5
    w = 0
    for gam in range(LL.shape[0]):
        Q, g = divmod(gam, s.nchol)

        def f(e):
            M = Af.conj().T @ scipy.linalg.expm(e * LL[gam]) @ U[w]
            sgn, la = np.linalg.slogdet(M)
            return 2.0 * (la + 1j * np.angle(sgn))

        fd = (f(eps) - f(-eps)) / (2 * eps)
        assert abs(fd - X[w, Q, g]) < 1e-7 * max(1.0, abs(X[w, Q, g]))


# ---------------------------------------------------------------------------
# P-4: Hartree identity links force bias and Coulomb energy
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mesh", [(2, 2, 2), (3, 1, 1), (1, 2, 3)])
def test_hartree_identity(mesh):
    s, U, _ = tiny(mesh, trial="random")
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    Gh, _ = kp.greens(U, s.A)
    xbar, _ = kp.force_bias(pre["Lh"], Gh, mesh, s.dt)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, mesh)
    hart = -np.sum(xbar ** 2, axis=(1, 2, 3)) / (2.0 * s.dt)
    assert np.abs(E[:, 1] - hart).max() < 1e-11 * max(1.0, np.abs(hart).max())


# ---------------------------------------------------------------------------
# P-5: the HS exponent is anti-Hermitian for real fields (unitary propagator)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mesh", [(2, 2, 2), (3, 1, 1), (2, 3, 1)])
def test_hs_exponent_antihermitian(mesh):
    s, U, x = tiny(mesh, trial="random")
    zeta = kp.combined_field(x, np.zeros_like(x, dtype=complex), mesh)
    vhs = kp.hs_potential(s.L, zeta, mesh)
    V = -math.sqrt(s.dt) * vhs
    for w in range(V.shape[0]):
        assert np.abs(V[w] + V[w].conj().T).max() < 1e-15
        nv = np.linalg.norm(V[w], 2)
        T = kp.taylor_exp_apply(V[w], np.eye(V.shape[1]), 6)
        bound = nv ** 7 / math.factorial(7) * math.exp(nv)
        dev = np.linalg.norm(T.conj().T @ T - np.eye(V.shape[1]), 2)
        # T^H T - I = -(e^V)^H R - R^H e^V + R^H R with ||R|| <= bound
        assert dev <= 2.0 * bound + bound ** 2 + 1e-14


# ---------------------------------------------------------------------------
# P-6: 6th-order Taylor against scipy expm, within the remainder bound
# ---------------------------------------------------------------------------

def test_taylor_against_expm_bound():
    s, U, x = tiny((2, 2, 2), m=4, nocc=2, nchol=5, trial="random")
    rng = np.random.default_rng(3)
    for scale in (0.05, 0.5, 2.0):
        V = scale * (rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8)))
        Uw = U[0][:8]
        nv = np.linalg.norm(V, 2)
        err = np.linalg.norm(kp.taylor_exp_apply(V, Uw, 6) - scipy.linalg.expm(V) @ Uw, 2)
        bound = nv ** 7 / math.factorial(7) * math.exp(nv) * np.linalg.norm(Uw, 2)
        assert err <= bound * (1 + 1e-12) + 1e-14


# ---------------------------------------------------------------------------
# P-7: Nk = 1 reduces to the standard (molecular) representation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("trial", ["identity", "random"])
def test_nk1_reduces_to_standard_representation(trial):
    s, U, x = tiny((1, 1, 1), m=6, nocc=3, nchol=9, trial=trial, nw=3)
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    Gh, _ = kp.greens(U, s.A)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    xbar, _ = kp.force_bias(pre["Lh"], Gh, s.mesh, s.dt)
    for w in range(U.shape[0]):
        Em = mol.energy_standard(s.L[0, 0], s.H1[0], s.A[0], Gh[w])
        assert np.abs(E[w] - Em).max() < 1e-12 * max(1.0, np.abs(Em).max())
        xm = mol.force_bias_standard(s.L[0, 0], s.A[0], Gh[w], s.dt)
        assert np.abs(xbar[w, 0] - xm).max() < 1e-14
        # self-inverse Q: no (-) component
        assert np.abs(xbar[w, :, :, 1]).max() < 1e-15


# ---------------------------------------------------------------------------
# P-8: k-block-diagonal walkers
# ---------------------------------------------------------------------------

def test_block_diagonal_walker_special_cases():
    mesh = (2, 3, 1)
    s, U, _ = tiny(mesh, m=5, nocc=2, nchol=4, trial="identity", walkers="blockdiag")
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    Gh, _ = kp.greens(U, s.A)
    Gb = Gh.reshape(U.shape[0], s.nk, s.nocc, s.nk, s.m)
    for k1 in range(s.nk):
        for k2 in range(s.nk):
            if k1 != k2:
                assert np.abs(Gb[:, k1, :, k2, :]).max() == 0.0
    xbar, X = kp.force_bias(pre["Lh"], Gh, mesh, s.dt)
    assert np.abs(X[:, 1:, :]).max() == 0.0
    _, negq = kp.kpoint_tables(mesh)
    for Q in range(s.nk):
        if negq[Q] == Q:
            assert np.abs(xbar[:, Q, :, 1]).max() == 0.0


# ---------------------------------------------------------------------------
# P-9: blocked formulas = unfolded supercell for every quantity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mesh", MESHES)
def test_blocked_equals_supercell(mesh):
    s, U, x = tiny(mesh, m=4, nocc=2, nchol=5, trial="random", walkers="dense")
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    LL, v, h, Af = supercell_objects(s)
    Gh, logdet = kp.greens(U, s.A)
    xbar, _ = kp.force_bias(pre["Lh"], Gh, mesh, s.dt)
    zeta = kp.combined_field(x, xbar, mesh)
    vhs = kp.hs_potential(s.L, zeta, mesh)
    U2 = kp.propagate(U, vhs, pre["bhalf"], s.dt)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, mesh)
    D = kp.energy_gradient(pre["Lh"], pre["h1h"], Gh, mesh)
    V0 = sc.v0_full(LL)
    assert np.abs(V0 - sc.block_diag(pre["V0"])).max() < 1e-13
    Bfull = scipy.linalg.expm(-0.5 * s.dt * (h + V0))
    assert np.abs(Bfull - sc.block_diag(pre["bhalf"])).max() < 1e-13
    for w in range(U.shape[0]):
        assert np.abs(sc.half_greens_full(U[w], Af) - Gh[w]).max() < 1e-12
        G = sc.greens_full(U[w], Af)
        xb1 = sc.force_bias_full(LL, G, s.dt).reshape(s.nk, s.nchol, 2)
        assert np.abs(xb1 - xbar[w]).max() < 1e-14
        V1 = sc.hs_matrix_full(LL, x[w].reshape(-1, 2), xbar[w].reshape(-1, 2), s.dt)
        assert np.abs(V1 + math.sqrt(s.dt) * vhs[w]).max() < 1e-15
        Up = sc.propagate_full(U[w], V1, h, V0, s.dt)
        assert np.abs(Up - U2[w]).max() < 1e-13
        E1 = sc.energy_4index(h, v, G)
        assert np.abs(E1 - E[w]).max() < 1e-12 * max(1.0, np.abs(E1).max())
        F = sc.fock(h, v, G)
        assert np.abs(2.0 * Af.conj().T @ F - D[w]).max() < 1e-12 * max(1.0, np.abs(D[w]).max())
    # weights (importance function and phaseless cut) against routes that share nothing with
    # the oracle's LU log determinants: the overlap ratio (det O'/det O)^2 from the
    # eigenvalues of the supercell overlap matrices, and the Gaussian factor as the ratio of
    # normal densities p(x - xbar) / p(x), continued to complex xbar
    w0 = np.array([1.0, 0.5])[: U.shape[0]]
    _, logdet2 = kp.greens(U2, s.A)
    w_or, log_I, dth = kp.weight_update(logdet, logdet2, x, xbar, w0)
    for w in range(U.shape[0]):
        ev0 = np.linalg.eigvals(Af.conj().T @ U[w])
        ev1 = np.linalg.eigvals(Af.conj().T @ U2[w])
        ratio = np.prod(ev1 / ev0) ** 2
        dens = np.exp(-0.5 * (x[w] - xbar[w]) ** 2) / np.exp(-0.5 * x[w] ** 2)
        imp = ratio * np.prod(dens)
        assert abs(np.exp(log_I[w]) / imp - 1.0) < 1e-11
        assert abs(dth[w] - np.angle(ratio)) < 1e-11
        assert abs(w_or[w] - abs(imp) * max(0.0, math.cos(np.angle(ratio))) * w0[w]) \
            < 1e-11 * w_or[w] + 1e-300


def test_importance_factor_is_density_ratio():
    """For real force biases the Gaussian part of the importance function,
    exp(sum x xbar - xbar^2/2), is the ratio of standard normal densities p(x - xbar)/p(x):
    the shifted sampling density over the unshifted one."""
    from scipy.stats import norm
    rng = np.random.default_rng(5)
    x = rng.standard_normal((3, 2, 4, 2))
    xbar = 0.3 * rng.standard_normal(x.shape)
    zero = np.zeros(3, dtype=complex)
    w, log_I, dth = kp.weight_update(zero, zero, x, xbar.astype(complex), np.ones(3))
    ref = np.prod(norm.pdf(x - xbar) / norm.pdf(x), axis=(1, 2, 3))
    np.testing.assert_allclose(w, ref, rtol=1e-12)
    np.testing.assert_allclose(log_I.real, np.log(ref), rtol=1e-12)
    assert np.all(dth == 0.0)


# ---------------------------------------------------------------------------
# P-10: adjoint = exact central difference (E is quadratic in Gh)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mesh", [(2, 2, 2), (2, 3, 1)])
def test_adjoint_exact_central_difference(mesh):
    s, U, _ = tiny(mesh, trial="random")
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    Gh, _ = kp.greens(U, s.A)
    D = kp.energy_gradient(pre["Lh"], pre["h1h"], Gh, mesh)
    rng = np.random.default_rng(7)
    for _ in range(3):
        dl = rng.standard_normal(Gh.shape) + 1j * rng.standard_normal(Gh.shape)
        h = 1e-3  # quadratic: no truncation error at any step
        Ep = kp.local_energy(pre["Lh"], pre["h1h"], Gh + h * dl, mesh).sum(1)
        Em = kp.local_energy(pre["Lh"], pre["h1h"], Gh - h * dl, mesh).sum(1)
        fd = (Ep - Em) / (2 * h)
        an = np.sum(D * dl, axis=(1, 2))
        assert np.abs(fd - an).max() < 1e-9 * max(1.0, np.abs(an).max())
    # entrywise on one walker, a few entries
    for (i, j) in [(0, 0), (1, 3), (Gh.shape[1] - 1, Gh.shape[2] - 1)]:
        e = np.zeros_like(Gh)
        e[0, i, j] = 1.0
        h = 1e-6
        Ep = kp.local_energy(pre["Lh"], pre["h1h"], Gh + h * e, mesh)[0].sum()
        Em = kp.local_energy(pre["Lh"], pre["h1h"], Gh - h * e, mesh)[0].sum()
        assert abs((Ep - Em) / (2 * h) - D[0, i, j]) < 1e-6 * max(1.0, abs(D[0, i, j]))


def test_adjoint_at_trial_is_fock_matrix():
    s, _, _ = tiny((2, 2, 2), m=4, nocc=2, nchol=5, trial="identity")
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    _, v, h, Af = supercell_objects(s)
    Gh, _ = kp.greens(Af[None], s.A)
    D = kp.energy_gradient(pre["Lh"], pre["h1h"], Gh, s.mesh)[0]
    # at the trial, G is the projector onto the occupied orbitals
    P = Af @ Af.conj().T
    F = sc.fock(h, v, P.T)
    occ = [k * s.m + a for k in range(s.nk) for a in range(s.nocc)]
    assert np.abs(D - 2.0 * F[occ, :]).max() < 1e-12


# ---------------------------------------------------------------------------
# orthonormalisation and weights
# ---------------------------------------------------------------------------

def test_orthonormalize_preserves_g_and_energy():
    mesh = (2, 3, 1)
    s, U, x = tiny(mesh, trial="random")
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    Ub = U * 3.0 + 0.5 * np.roll(U, 1, axis=2)
    Q = kp.orthonormalize(Ub)
    for w in range(U.shape[0]):
        assert np.abs(Q[w].conj().T @ Q[w] - np.eye(U.shape[2])).max() < 1e-13
        R = Q[w].conj().T @ Ub[w]
        assert np.abs(np.tril(R, -1)).max() < 1e-12
        assert np.all(np.diag(R).real > 0) and np.abs(np.diag(R).imag).max() < 1e-12
    G1, _ = kp.greens(Ub, s.A)
    G2, _ = kp.greens(Q, s.A)
    assert np.abs(G1 - G2).max() < 1e-11


def test_weight_update_cases():
    nw = 4
    x = np.zeros((nw, 2, 3, 2))
    xbar = np.zeros_like(x, dtype=complex)
    ld0 = np.zeros(nw, dtype=complex)
    ld1 = np.array([0.1, 0.1 + 0.3j, 0.0 + 1.0j, -0.2 + 0.5j])
    w0 = np.array([1.0, 2.0, 1.0, 0.5])
    w1, logI, dth = kp.weight_update(ld0, ld1, x, xbar, w0)
    # ratio = exp(2 dlogdet); angle of ratio; cos cut
    np.testing.assert_allclose(dth, [0.0, 0.6, 2.0, 1.0], atol=1e-15)
    assert w1[2] == 0.0
    np.testing.assert_allclose(w1[0], math.exp(0.2), rtol=1e-15)
    np.testing.assert_allclose(w1[1], 2.0 * math.exp(0.2) * math.cos(0.6), rtol=1e-15)
    # importance factor with a force bias: exp(x xbar - xbar^2/2)
    x2 = np.full((1, 1, 1, 2), 0.5)
    xb2 = np.full((1, 1, 1, 2), 0.25 + 0.1j)
    w2, logI2, _ = kp.weight_update(np.zeros(1), np.zeros(1), x2, xb2, np.ones(1))
    s = 2 * (0.5 * (0.25 + 0.1j) - 0.5 * (0.25 + 0.1j) ** 2)
    np.testing.assert_allclose(logI2[0], s, rtol=1e-15)
    np.testing.assert_allclose(w2[0], math.exp(s.real), rtol=1e-15)


# ---------------------------------------------------------------------------
# mixed estimate of the energy
# ---------------------------------------------------------------------------

def test_mixed_energy_cases():
    E = np.array([[1.0, 2.0, -0.5], [2.0 + 1.0j, 0.0, 0.0], [10.0, 0.0, 0.0]])
    EL = E.sum(1)
    # equal weights: the plain mean; a zero weight drops its walker
    assert abs(kp.mixed_energy(E, np.ones(3)) - EL.mean()) < 1e-15
    assert abs(kp.mixed_energy(E, [1.0, 1.0, 0.0]) - EL[:2].mean()) < 1e-15
    # weights are relative: scaling them changes nothing
    w = np.array([0.3, 1.7, 2.0])
    assert abs(kp.mixed_energy(E, w) - kp.mixed_energy(E, 5.0 * w)) < 1e-14
    assert abs(kp.mixed_energy(E, w) - (w * EL).sum() / w.sum()) < 1e-15


def test_mixed_energy_on_trial_walkers_is_slater_condon():
    """Walkers on the trial determinant: the mixed estimate is the HF energy from explicit
    4-index integrals, for any weights."""
    s, _, _ = tiny((2, 2, 2), m=4, nocc=2, nchol=5, trial="random")
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    LL, v, h, Af = supercell_objects(s)
    Gh, _ = kp.greens(np.stack([Af, Af, Af]), s.A)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    e_hf = sum(sc.slater_condon_energy(h, v, Af))
    assert abs(kp.mixed_energy(E, [0.2, 3.0, 1.0]) - e_hf) < 1e-11 * max(1.0, abs(e_hf))


# ---------------------------------------------------------------------------
# population control (comb): properties any correct comb has
# ---------------------------------------------------------------------------

from oracle import walkers as wk


def test_comb_worked_example():
    # cumulative weights 0.5, 2.0, 2.0, 4.0; points 0.25, 1.25, 2.25, 3.25 (spacing 1)
    par = wk.comb_parents([0.5, 1.5, 0.0, 2.0], 0.25)
    assert par.tolist() == [0, 1, 3, 3]
    # the point 2.0 lies on the boundary after the empty interval of walker 2
    assert wk.comb_parents([0.5, 1.5, 0.0, 2.0], 0.0).tolist() == [0, 1, 3, 3]
    assert wk.comb_parents([1.0, 0.0, 0.0, 3.0], 0.5).tolist() == [0, 3, 3, 3]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_comb_copy_counts_are_floor_or_ceiling(seed):
    rng = np.random.default_rng(seed)
    W = 64
    w = rng.exponential(size=W)
    w[rng.choice(W, 9, replace=False)] = 0.0
    for xi in rng.random(20):
        par = wk.comb_parents(w, xi)
        n = np.bincount(par, minlength=W)
        expect = W * w / w.sum()
        assert n.sum() == W
        assert np.all(n >= np.floor(expect) - 1e-12) and np.all(n <= np.ceil(expect) + 1e-12)
        assert np.all(n[w == 0] == 0)
        assert np.all(np.diff(par) >= 0)  # copies come out in walker order


def test_comb_unbiased_over_xi():
    rng = np.random.default_rng(7)
    W = 16
    w = rng.exponential(size=W)
    S = 4000
    n = np.zeros(W)
    for s in range(S):
        n += np.bincount(wk.comb_parents(w, (s + 0.5) / S), minlength=W)
    # the midpoint rule in xi is exact up to one point per interval boundary crossing
    assert np.allclose(n / S, W * w / w.sum(), atol=2.0 / S)


def test_comb_identity_and_degenerate_cases():
    W = 10
    for xi in (0.0, 0.3, 0.999):
        assert wk.comb_parents(np.full(W, 2.5), xi).tolist() == list(range(W))
    assert wk.comb_parents(np.zeros(W), 0.4).tolist() == list(range(W))
    bad = np.ones(W)
    bad[3] = -1.0
    assert wk.comb_parents(bad, 0.4).tolist() == list(range(W))
    bad[3] = np.nan
    assert wk.comb_parents(bad, 0.4).tolist() == list(range(W))
    one = np.zeros(W)
    one[6] = 1e-300
    assert wk.comb_parents(one, 0.999999).tolist() == [6] * W


def test_population_control_state():
    rng = np.random.default_rng(3)
    W = 8
    U = rng.normal(size=(W, 5, 2)) + 1j * rng.normal(size=(W, 5, 2))
    G = rng.normal(size=(W, 2, 5)) + 0j
    ld = rng.normal(size=W) + 1j * rng.normal(size=W)
    st = np.arange(W, dtype=np.int32)
    w = rng.exponential(size=W)
    U2, G2, ld2, st2, w2, par = wk.population_control(U, G, ld, st, w, 0.6)
    assert np.array_equal(U2, U[par]) and np.array_equal(G2, G[par])
    assert np.array_equal(ld2, ld[par]) and np.array_equal(st2, st[par])
    assert np.allclose(w2, w.sum() / W) and np.isclose(w2.sum(), w.sum())


# ---------------------------------------------------------------------------
# Blocking analysis of block energies (oracle/blocking.py)
from oracle import blocking as blk  # noqa: E402


def test_reblock_worked_example():
    """x = 1, 2, 3, 4 by hand: level 0 mean 5/2, s^2 = 5/3, err = sqrt(5/12); level 1 the
    pair means 3/2 and 7/2, s^2 = 2, err = 1; no level 2 (one block)."""
    lv = blk.reblock([1.0, 2.0, 3.0, 4.0])
    assert len(lv) == 2
    n, mean, err, ee = lv[0]
    assert n == 4 and mean == 2.5
    assert err == pytest.approx(math.sqrt(5.0 / 12.0), rel=1e-15)
    assert ee == pytest.approx(math.sqrt(5.0 / 12.0) / math.sqrt(6.0), rel=1e-15)
    n, mean, err, ee = lv[1]
    assert n == 2 and mean == 2.5 and err == pytest.approx(1.0, rel=1e-15)
    # odd length: the last element is dropped when pairing
    lv = blk.reblock([1.0, 2.0, 3.0, 4.0, 100.0])
    assert lv[1][0] == 2 and lv[1][1] == 2.5


def test_reblock_iid_standard_error():
    """iid N(0, 1): every level estimates 1/sqrt(N), and the chosen level's error is within
    its statistical uncertainty of it."""
    rng = np.random.default_rng(7)
    N = 1 << 16
    lv = blk.reblock(rng.standard_normal(N))
    opt = blk.optimal_level(lv)
    assert opt >= 0
    _, _, err, ee = lv[opt]
    assert abs(err - 1.0 / math.sqrt(N)) < 4.0 * ee
    # B^3 > 2N with err ratio about 1: B = 2^opt is the first power of two past (2N)^(1/3)
    assert 2 ** (opt - 1) <= (2.0 * N) ** (1.0 / 3.0) * 1.5


def test_reblock_ar1_standard_error():
    """AR(1) x_t = phi x_{t-1} + e_t, e ~ N(0, 1): the variance of the mean of N terms is
    (1 / (1 - phi^2)) (1 + phi) / (1 - phi) / N for large N (the integrated autocorrelation
    time (1 + phi) / (1 - phi)); the chosen level recovers it, level 0 underestimates it by
    the factor sqrt((1 - phi) / (1 + phi))."""
    rng = np.random.default_rng(11)
    N, phi = 1 << 17, 0.8
    e = rng.standard_normal(N)
    x = np.empty(N)
    x[0] = e[0] / math.sqrt(1.0 - phi * phi)
    for t in range(1, N):
        x[t] = phi * x[t - 1] + e[t]
    true = math.sqrt((1.0 / (1.0 - phi * phi)) * (1.0 + phi) / (1.0 - phi) / N)
    lv = blk.reblock(x)
    opt = blk.optimal_level(lv)
    assert opt > 0
    _, _, err, ee = lv[opt]
    assert abs(err - true) < 4.0 * ee + 0.05 * true
    assert lv[0][2] < 0.5 * true


def test_reblock_shift_and_scale():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(1000)
    a, b = blk.reblock(x), blk.reblock(-3.0 * x + 17.0)
    assert len(a) == len(b)
    for (n1, m1, e1, _), (n2, m2, e2, _) in zip(a, b):
        assert n1 == n2
        assert m2 == pytest.approx(-3.0 * m1 + 17.0, abs=1e-12)
        assert e2 == pytest.approx(3.0 * e1, rel=1e-10)
    assert blk.optimal_level(a) == blk.optimal_level(b)
    assert blk.optimal_level([]) == -1
    assert blk.reblock([1.0]) == []


# ---------------------------------------------------------------------------
# Energy shift E_T of the projector exp(-dt (H - E_T))
# ---------------------------------------------------------------------------

def test_energy_shift_is_a_common_factor():
    """The shift multiplies every walker's new weight by exp(dt E_T) and changes nothing
    else: the walkers, the mixed estimate and the comb's parents are those without it."""
    s, _, _ = tiny((2, 1, 1), m=5, nocc=2, nchol=7, trial="random")
    rng = np.random.default_rng(5)
    U = make_walkers(s, 6, rng, kind="dense")
    x = make_fields(s, 6, 1, rng)[0]
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    _, ld = kp.greens(U, s.A)
    w0 = rng.uniform(0.5, 2.0, 6)
    a = kp.step(U, ld, w0, x, pre, s.A, s.L, s.mesh, s.dt)
    ET = -3.7
    b = kp.step(U, ld, w0, x, pre, s.A, s.L, s.mesh, s.dt, etrial=ET)
    assert np.array_equal(a["U"], b["U"]) and np.array_equal(a["Gh"], b["Gh"])
    np.testing.assert_allclose(b["weight"], a["weight"] * math.exp(s.dt * ET), rtol=1e-14)
    E = kp.local_energy(pre["Lh"], pre["h1h"], a["Gh"], s.mesh)
    assert abs(kp.mixed_energy(E, a["weight"]) - kp.mixed_energy(E, b["weight"])) < 1e-12
    for xi in (0.1, 0.6):
        assert np.array_equal(wk.comb_parents(a["weight"], xi), wk.comb_parents(b["weight"], xi))


# ---------------------------------------------------------------------------
# The standard (dense) representation of a k-point system (oracle/dense.py)
from oracle import dense as dn  # noqa: E402


def _dense_system(s):
    Ld = dn.dense_cholesky(s.L, s.mesh)
    H1d, Ad = dn.dense_one_body(s.H1, s.A)
    return Ld, H1d, Ad


@pytest.mark.parametrize("mesh", [(2, 1, 1), (3, 1, 1), (2, 3, 1), (1, 2, 3)])
def test_dense_vectors_reproduce_integrals(mesh):
    """The dense vectors are Hermitian and give the explicit 4-index integrals and V0 of the
    unfolded k-point operators; their number is Nk C."""
    s, _, _ = tiny(mesh, m=3, nocc=1, nchol=4)
    Ld, _, _ = _dense_system(s)
    N = s.nk * s.m
    assert Ld.shape == (1, 1, N, N, s.nk * s.nchol)
    D = Ld[0, 0].transpose(2, 0, 1)  # [g, P, R]
    assert np.abs(D - D.conj().transpose(0, 2, 1)).max() < 1e-15
    LL = sc.unfold_cholesky(s.L, s.mesh)
    assert np.abs(sc.eri(D) - sc.eri(LL)).max() < 1e-13
    assert np.abs(sc.v0_full(D) - sc.v0_full(LL)).max() < 1e-13


@pytest.mark.parametrize("mesh", [(2, 1, 1), (3, 1, 1), (2, 3, 1)])
def test_dense_energy_and_step_equal_kpoint(mesh):
    """The same walkers in both representations: equal local energies, and one step with the
    mapped fields gives the same walkers, log overlaps and weights."""
    s, U, x = tiny(mesh, m=4, nocc=2, nchol=5, nw=3)
    Ld, H1d, Ad = _dense_system(s)
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    pred = kp.prepare(Ld, H1d, Ad, s.dt)
    Gh, ld = kp.greens(U, s.A)
    Ghd, ldd = kp.greens(U, Ad)
    assert np.abs(Gh - Ghd).max() < 1e-12
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, s.mesh)
    Ed = kp.local_energy(pred["Lh"], pred["h1h"], Ghd, (1, 1, 1))
    assert np.abs(E.sum(1) - Ed.sum(1)).max() < 1e-11 * np.abs(E).sum(1).max()
    # E1B agrees part by part; the two-body parts only in total (the dense EC takes what the
    # k-point exchange of Q != 0 pairs carries in its direct term and vice versa)
    assert np.abs(E[:, 0] - Ed[:, 0]).max() < 1e-12 * np.abs(E[:, 0]).max()
    xd = dn.dense_fields(x, s.mesh)
    w = np.ones(U.shape[0])
    a = kp.step(U, ld, w, x, pre, s.A, s.L, s.mesh, s.dt)
    b = kp.step(U, ldd, w, xd, pred, Ad, Ld, (1, 1, 1), s.dt)
    assert np.abs(a["U"] - b["U"]).max() < 1e-12
    np.testing.assert_allclose(b["weight"], a["weight"], rtol=1e-12)
    assert np.abs(np.exp(a["logdet"] - b["logdet"]) - 1).max() < 1e-12


# ---------------------------------------------------------------------------
# collinear (two-determinant) walkers
# ---------------------------------------------------------------------------

from synth import make_spin_trial, spin_view  # noqa: E402
from oracle import spin as sp  # noqa: E402


def spin_case(mesh, m=4, n_up=2, n_dn=1, nchol=5, nw=2, seed=21, walkers="dense"):
    s, rng = make_system(mesh, m, n_up, nchol, seed=seed, trial="random")
    A_dn = make_spin_trial(s, n_dn, rng)
    U_up = make_walkers(s, nw, rng, kind=walkers)
    U_dn = make_walkers(spin_view(s, A_dn), nw, rng, kind=walkers)
    x = make_fields(s, nw, 1, rng)[0]
    return s, (s.A, A_dn), (U_up, U_dn), x


@pytest.mark.parametrize("mesh", [(1, 1, 1), (2, 1, 1), (2, 3, 1), (2, 2, 2)])
def test_spin_equal_spins_reduce_to_closed_shell(mesh):
    """Equal up and down determinants: the closed-shell energy, force bias and weights, and
    each spin's gradient is half the closed-shell one (E_cs(G) = E(G, G))."""
    s, U, x = tiny(mesh, trial="random")
    pre = kp.prepare(s.L, s.H1, s.A, s.dt)
    ps = sp.prepare(s.L, s.H1, s.A, s.A, s.dt)
    Gh, ld = kp.greens(U, s.A)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, mesh)
    Es = sp.local_energy(ps["Lh"], ps["h1h"], (Gh, Gh), mesh)
    assert np.abs(Es - E).max() < 1e-12 * np.abs(E).max()
    xb, X = kp.force_bias(pre["Lh"], Gh, mesh, s.dt)
    xbs, Xs = sp.force_bias(ps["Lh"], (Gh, Gh), mesh, s.dt)
    assert np.abs(xbs - xb).max() < 1e-14 and np.abs(Xs - X).max() < 1e-13
    g = kp.energy_gradient(pre["Lh"], pre["h1h"], Gh, mesh)
    gu, gd = sp.energy_gradient(ps["Lh"], ps["h1h"], (Gh, Gh), mesh)
    assert np.abs(gu - 0.5 * g).max() < 1e-13 and np.abs(gd - 0.5 * g).max() < 1e-13
    w0 = np.array([1.0, 0.7])
    r = kp.step(U, ld, w0, x, pre, s.A, s.L, mesh, s.dt, etrial=-1.5)
    rs = sp.step((U, U), (ld, ld), w0, x, ps, (s.A, s.A), s.L, mesh, s.dt, etrial=-1.5)
    for q in range(2):
        assert np.abs(rs["U"][q] - r["U"]).max() < 1e-14
        assert np.abs(rs["logdet"][q] - r["logdet"]).max() < 1e-13
    np.testing.assert_allclose(rs["weight"], r["weight"], rtol=1e-13)


@pytest.mark.parametrize("mesh", [(1, 1, 1), (2, 1, 1), (2, 3, 1), (1, 1, 2)])
@pytest.mark.parametrize("nocc", [(2, 1), (1, 2), (2, 2), (3, 0)])
def test_spin_energy_equals_4index(mesh, nocc):
    """The energy of two different determinants against the spin-resolved expression with
    explicit supercell integrals (Hamiltonian of "Introduction to AFQMC", Wick's theorem):
    E = sum_s sum h_PQ G^s_PQ + 1/2 sum v_PQRS [(G^u + G^d)_PR (G^u + G^d)_QS
                                               - sum_s G^s_PS G^s_QR]."""
    n_up, n_dn = nocc
    s, A, U, _ = spin_case(mesh, m=4, n_up=n_up, n_dn=max(n_dn, 1))
    if n_dn == 0:  # no down electrons: an empty determinant (Gh with zero rows, overlap 1)
        A = (A[0], A[1][:, :, :0])
        U = (U[0], U[1][:, :, :0])
    ps = sp.prepare(s.L, s.H1, A[0], A[1], s.dt)
    Gh = tuple(kp.greens(U[q], A[q])[0] for q in range(2))
    E = sp.local_energy(ps["Lh"], ps["h1h"], Gh, mesh)
    LL, v, h, _ = supercell_objects(s)
    for w in range(U[0].shape[1] and U[0].shape[0]):
        G = []
        for q in range(2):
            Af = sc.block_diag(A[q])
            G.append(sc.greens_full(U[q][w], Af) if A[q].shape[2] else np.zeros_like(h))
        Gt = G[0] + G[1]
        e1 = sum(np.sum(h * G[q]) for q in range(2))
        ec = 0.5 * np.einsum("pqrs,pr,qs->", v, Gt, Gt, optimize=True)
        ex = -0.5 * sum(np.einsum("pqrs,ps,qr->", v, G[q], G[q], optimize=True)
                        for q in range(2))
        ref = np.array([e1, ec, ex])
        assert np.abs(E[w] - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_spin_energy_swap_and_force_bias_derivative():
    """Swapping the spins leaves energy and force bias unchanged; the force bias is the
    derivative of the log of the two-determinant overlap."""
    mesh = (2, 3, 1)
    s, A, U, _ = spin_case(mesh, m=3, n_up=2, n_dn=1, nchol=3)
    ps = sp.prepare(s.L, s.H1, A[0], A[1], s.dt)
    pw = sp.prepare(s.L, s.H1, A[1], A[0], s.dt)
    Gh = tuple(kp.greens(U[q], A[q])[0] for q in range(2))
    E = sp.local_energy(ps["Lh"], ps["h1h"], Gh, mesh)
    Ew = sp.local_energy(pw["Lh"], pw["h1h"], Gh[::-1], mesh)
    assert np.abs(E - Ew).max() < 1e-13 * np.abs(E).max()
    _, X = sp.force_bias(ps["Lh"], Gh, mesh, s.dt)
    LL, _, _, _ = supercell_objects(s)
    Af = [sc.block_diag(A[q]) for q in range(2)]
    eps = 1e-5
    w = 1
    for gam in range(LL.shape[0]):
        Q, g = divmod(gam, s.nchol)

        def f(e):
            out = 0.0
            for q in range(2):
                M = Af[q].conj().T @ scipy.linalg.expm(e * LL[gam]) @ U[q][w]
                sgn, la = np.linalg.slogdet(M)
                out = out + la + 1j * np.angle(sgn)
            return out

        fd = (f(eps) - f(-eps)) / (2 * eps)
        assert abs(fd - X[w, Q, g]) < 1e-7 * max(1.0, abs(X[w, Q, g]))


def test_spin_gradient_finite_difference():
    """The per-spin adjoint against central differences of the energy (a quadratic
    polynomial in Gh: the difference is exact up to rounding)."""
    mesh = (2, 1, 1)
    s, A, U, _ = spin_case(mesh, m=4, n_up=2, n_dn=1, nchol=4)
    ps = sp.prepare(s.L, s.H1, A[0], A[1], s.dt)
    Gh = tuple(kp.greens(U[q], A[q])[0] for q in range(2))
    g = sp.energy_gradient(ps["Lh"], ps["h1h"], Gh, mesh)
    rng = np.random.default_rng(7)
    for q in range(2):
        D = rng.standard_normal(Gh[q].shape) + 1j * rng.standard_normal(Gh[q].shape)
        eps = 1e-3

        def E(e):
            G2 = list(Gh)
            G2[q] = Gh[q] + e * D
            return sp.local_energy(ps["Lh"], ps["h1h"], tuple(G2), mesh).sum(axis=1)

        fd = (E(eps) - E(-eps)) / (2 * eps)
        an = np.einsum("wij,wij->w", g[q], D)
        assert np.abs(fd - an).max() < 1e-9 * max(1.0, np.abs(an).max())


def test_spin_step_overlap_ratio_dense():
    """One step of different up and down determinants: each spin's walker is the dense
    supercell propagator applied to it, and the weight's overlap ratio is the product of the
    two spins' dense determinant ratios."""
    mesh = (2, 1, 1)
    s, A, U, x = spin_case(mesh, m=4, n_up=2, n_dn=1, nchol=4)
    ps = sp.prepare(s.L, s.H1, A[0], A[1], s.dt)
    ld = tuple(kp.greens(U[q], A[q])[1] for q in range(2))
    w0 = np.array([1.0, 2.0])
    r = sp.step(U, ld, w0, x, ps, A, s.L, mesh, s.dt)
    LL, _, h, _ = supercell_objects(s)
    V0 = sc.v0_full(LL)
    for w in range(2):
        V = sc.hs_matrix_full(LL, x[w].reshape(-1, 2), r["xbar"][w].reshape(-1, 2), s.dt)
        ratio = 1.0
        for q in range(2):
            Af = sc.block_diag(A[q])
            Un = sc.propagate_full(U[q][w], V, h, V0, s.dt)
            assert np.abs(r["U"][q][w] - Un).max() < 1e-13
            ratio *= np.linalg.det(Af.conj().T @ Un) / np.linalg.det(Af.conj().T @ U[q][w])
        log_r = r["log_I"][w] - np.sum(x[w] * r["xbar"][w] - 0.5 * r["xbar"][w] ** 2)
        assert abs(np.exp(log_r) / ratio - 1.0) < 1e-12


# ---------------------------------------------------------------------------
# non-uniform band counts: the zero-padded uniform system is the ragged system
# ---------------------------------------------------------------------------

from synth import make_ragged_system, make_ragged_walkers  # noqa: E402
from oracle import bands as bd  # noqa: E402

RAGGED = [((2, 1, 1), (4, 6)), ((2, 3, 1), (4, 5, 3, 4, 6, 5)), ((1, 1, 2), (5, 3)),
          ((2, 2, 1), (3, 5, 4, 4))]


@pytest.mark.parametrize("mesh,mk", RAGGED)
def test_padded_bands_equal_supercell(mesh, mk):
    """Energy, force bias, one step (walkers, log overlaps, weights) of the padded system
    against the supercell route of the ragged system, which knows nothing of padding."""
    rs, rng = make_ragged_system(mesh, mk, 2, 5, seed=4)
    Ur = make_ragged_walkers(rs, 2, rng)
    x = rng.standard_normal((2, rs.nk, rs.nchol, 2))
    m = max(mk) + 1  # one band of padding beyond the largest count
    L, H1, A = bd.pad(rs, m)
    U = bd.pad_walkers(Ur, mk, m)
    assert np.array_equal(bd.unpad_walkers(U, mk, m), Ur)
    pre = kp.prepare(L, H1, A, rs.dt)
    Gh, ld = kp.greens(U, A)
    E = kp.local_energy(pre["Lh"], pre["h1h"], Gh, mesh)
    xbar, _ = kp.force_bias(pre["Lh"], Gh, mesh, rs.dt)
    r = kp.step(U, ld, np.ones(2), x, pre, A, L, mesh, rs.dt)
    LL, h, Af = bd.supercell(rs)
    v = sc.eri(LL)
    V0 = sc.v0_full(LL)
    for w in range(2):
        assert np.abs(bd.unpad_greens(Gh, mk, m)[w] - sc.half_greens_full(Ur[w], Af)).max() \
            < 1e-12
        G = sc.greens_full(Ur[w], Af)
        ref = sc.energy_4index(h, v, G)
        assert np.abs(E[w] - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
        xb = sc.force_bias_full(LL, G, rs.dt).reshape(rs.nk, rs.nchol, 2)
        assert np.abs(xbar[w] - xb).max() < 1e-14
        V = sc.hs_matrix_full(LL, x[w].reshape(-1, 2), xb.reshape(-1, 2), rs.dt)
        Un = sc.propagate_full(Ur[w], V, h, V0, rs.dt)
        assert np.abs(bd.unpad_walkers(r["U"], mk, m)[w] - Un).max() < 1e-13
        # the padded rows stay zero
        pad_rows = np.ones(rs.nk * m, dtype=bool)
        for k in range(rs.nk):
            pad_rows[k * m:k * m + mk[k]] = False
        assert np.abs(r["U"][w][pad_rows]).max() < 1e-15
        ratio = np.linalg.det(Af.conj().T @ Un) / np.linalg.det(Af.conj().T @ Ur[w])
        assert abs(np.exp(r["logdet"][w] - ld[w]) / ratio - 1.0) < 1e-11
