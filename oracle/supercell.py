"""Brute force on the unfolded supercell (test infrastructure only).

Only tests, the repository smoke check and the benchmark's CPU-baseline leg
may import this module.

Everything here uses dense (nk*m)-dimensional matrices and, for the energy,
explicit 4-index integrals, following the generic (non-k-point) equations of
the standard representation: the Cholesky factorisation of the ERIs, the
Hubbard-Stratonovich potentials L+/- with their phases, the force bias, the
HS matrix, the Green's function and the local energy.  It is meant for tiny
meshes, where it pins the blocked k-point formulas.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg


def _lin(v, mesh):
    v = [int(v[i]) % mesh[i] for i in range(3)]
    return (v[0] * mesh[1] + v[1]) * mesh[2] + v[2]


def _vec(k, mesh):
    return (k // (mesh[1] * mesh[2]), (k // mesh[2]) % mesh[1], k % mesh[2])


def unfold_cholesky(L, mesh):
    """Dense supercell operators LL[(Q g), P, R]; block (k, k - Q) of (Q, g) is L[Q][k][:, :, g].

    The momentum convention of the k-point Hamiltonian: the second band index
    of L^{Q,k} sits at k - Q.
    """
    nk, _, m, _, nchol = L.shape
    N = nk * m
    LL = np.zeros((nk, nchol, N, N), dtype=np.complex128)
    for Q in range(nk):
        qv = _vec(Q, mesh)
        for k in range(nk):
            kv = _vec(k, mesh)
            k2 = _lin([kv[i] - qv[i] for i in range(3)], mesh)
            LL[Q, :, k * m:(k + 1) * m, k2 * m:(k2 + 1) * m] = L[Q, k].transpose(2, 0, 1)
    return LL.reshape(nk * nchol, N, N)


def eri(LL):
    """v[P, Q, R, S] = sum_gamma LL[gamma, P, R] conj(LL[gamma, S, Q])."""
    ng, N, _ = LL.shape
    a = LL.reshape(ng, N * N)  # [gamma, (P R)]
    b = LL.conj().transpose(0, 2, 1).reshape(ng, N * N)  # [gamma, (Q S)] from conj(LL[g, S, Q])
    v = (a.T @ b).reshape(N, N, N, N)  # [P, R, Q, S]
    return v.transpose(0, 2, 1, 3)


def block_diag(blocks):
    """Dense block-diagonal matrix from blocks[k] (same shape each)."""
    nk, r, c = blocks.shape
    out = np.zeros((nk * r, nk * c), dtype=np.complex128)
    for k in range(nk):
        out[k * r:(k + 1) * r, k * c:(k + 1) * c] = blocks[k]
    return out


def greens_full(U, Afull):
    """G_PR = [A^* (U^T A^*)^{-1} U^T]_PR (spin-resolved Green's function of one spin)."""
    Ast = Afull.conj()
    return Ast @ np.linalg.inv(U.T @ Ast) @ U.T


def half_greens_full(U, Afull):
    """Gh = (U^T A^*)^{-1} U^T."""
    Ast = Afull.conj()
    return np.linalg.inv(U.T @ Ast) @ U.T


def energy_4index(h, v, G):
    """Closed-shell local energy from the generic expression with explicit integrals.

    E = sum_sigma sum h_PQ G_PQ
        + 1/2 sum_{sigma sigma'} v_PQRS (G_PR G'_QS - delta G_PS G_QR),
    with both spins equal: E1B = 2 sum h G, EC = 2 sum v G_PR G_QS,
    EX = -sum v G_PS G_QR.
    """
    E1 = 2.0 * np.sum(h * G)
    EC = 2.0 * np.einsum("pqrs,pr,qs->", v, G, G, optimize=True)
    EX = -np.einsum("pqrs,ps,qr->", v, G, G, optimize=True)
    return np.array([E1, EC, EX])


def slater_condon_energy(h, v, Afull):
    """<Psi_T|H|Psi_T> for a closed-shell determinant with orthonormal columns Afull.

    Textbook Slater-Condon rules in the orbital basis of the trial:
    E = 2 sum_a h_aa + 2 sum_ab v_abab - sum_ab v_abba,
    with h_ab = (A^H h A)_ab and v_abcd = sum conj(A_Pa) conj(A_Qb) A_Rc A_Sd v_PQRS.
    """
    hm = Afull.conj().T @ h @ Afull
    vm = np.einsum("pa,qb,rc,sd,pqrs->abcd", Afull.conj(), Afull.conj(), Afull, Afull, v,
                   optimize=True)
    n = Afull.shape[1]
    Ed = 2.0 * np.trace(hm)
    J = sum(vm[a, b, a, b] for a in range(n) for b in range(n))
    K = sum(vm[a, b, b, a] for a in range(n) for b in range(n))
    return Ed, 2.0 * J, -K


def fock(h, v, G):
    """Per-spin generalized Fock matrix F = h + J[2G] - K[G].

    J[D]_AB = sum_QS v_AQBS D_QS,  K[D]_AB = sum_QR v_AQRB D_QR.
    """
    J = np.einsum("aqbs,qs->ab", v, G, optimize=True)
    K = np.einsum("aqrb,qr->ab", v, G, optimize=True)
    return h + 2.0 * J - K


def hs_operators(LL):
    """L+ = (LL + LL^H)/2 and L- = (LL - LL^H)/2 per Cholesky vector."""
    LH = LL.conj().transpose(0, 2, 1)
    return 0.5 * (LL + LH), 0.5 * (LL - LH)


# phases of the two HS potentials: c+ = i, c- = 1 (anti-Hermitian v-hat)
C_PLUS = 1j
C_MINUS = 1.0


def force_bias_full(LL, G, dt):
    """xbar[gamma][+/-] = -sqrt(dt) c+/- sum_sigma sum_PR [L+/-]_PR G_PR (both spins)."""
    Lp, Lm = hs_operators(LL)
    sdt = np.sqrt(dt)
    xp = -sdt * C_PLUS * 2.0 * np.einsum("gpr,pr->g", Lp, G)
    xm = -sdt * C_MINUS * 2.0 * np.einsum("gpr,pr->g", Lm, G)
    return np.stack([xp, xm], axis=-1)


def hs_matrix_full(LL, x, xbar, dt):
    """V = sqrt(dt) sum_{gamma, +/-} c+/- [L+/-] (x - xbar): exponent of the two-body propagator."""
    Lp, Lm = hs_operators(LL)
    xt = x - xbar
    V = np.einsum("gpr,g->pr", Lp, C_PLUS * xt[:, 0]) + np.einsum("gpr,g->pr", Lm,
                                                                   C_MINUS * xt[:, 1])
    return np.sqrt(dt) * V


def v0_full(LL):
    """V0 = -1/2 sum_gamma LL LL^H (normal-ordering term)."""
    return -0.5 * np.einsum("gpr,gqr->pq", LL, LL.conj())


def propagate_full(U, V, h, V0, dt, order=6, exact=False):
    """Bhalf e^V Bhalf U with Bhalf = expm(-dt/2 (h + V0)); e^V by Taylor or scipy expm."""
    B = scipy.linalg.expm(-0.5 * dt * (h + V0))
    T = B @ U
    if exact:
        T = scipy.linalg.expm(V) @ T
    else:
        acc = T.copy()
        term = T
        for j in range(1, order + 1):
            term = V @ term / j
            acc = acc + term
        T = acc
    return B @ T
