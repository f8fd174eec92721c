"""Blocked k-point formulas of ph-AFQMC, FP64 (test infrastructure only).

Only tests, the repository smoke check and the benchmark's CPU-baseline leg
may import this module.  It shares no code with the GPU library.

Conventions (paper section "k-Point Representation")
----------------------------------------------------
* k is linearised row-major over the Monkhorst-Pack mesh; k - Q and -Q are
  componentwise mod mesh.
* L[Q][k][i][l][g]: Cholesky block with band i at k and band l at k - Q.  The
  supercell operator of (Q, g) has block (k, k - Q) equal to L[Q][k][:, :, g].
* Walkers U[w] are dense (nk*m) x (nk*nocc) matrices; the trial is block
  diagonal with blocks A[k] (m x nocc).
* Closed shell: one determinant for both spins.  Overlap = det(A^H U)^2.

Readings of points the text leaves open (each is listed with its reason in
the design notes of the repository):
* HS potentials use c+ = i, c- = 1 so that both are anti-Hermitian and the
  two-body propagator is unitary for real fields.
* The force bias carries the -sqrt(dt) factor of the standard form.
* The combined field of the single-contraction HS potential is
  xi_Q = 1/2 [ i (xt+_Q + xt+_-Q) + (xt-_Q - xt-_-Q) ], xt = x - xbar, and the
  exponent of the two-body propagator is sqrt(dt) * sum_Qg xi_Qg L_Qg.  The
  library's vhs is defined as -sum xi L, so the exponent reads -sqrt(dt) vhs.
* One-body propagator: Bhalf = exp(-dt/2 (H1 + V0)),
  V0 = -1/2 sum_{Q,g} L_Qg L_Qg^H (block diagonal in k).
* Taylor expansion of the two-body exponential to 6th order, term by term.
* Phaseless angle: the argument of the overlap ratio only.
"""

from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# index algebra
# ---------------------------------------------------------------------------

def kpoint_tables(mesh):
    """Return (kmq, negq): kmq[Q, k] = index of k - Q, negq[Q] = index of -Q."""
    mesh = tuple(int(v) for v in mesh)
    nk = mesh[0] * mesh[1] * mesh[2]
    vec = np.array([(k // (mesh[1] * mesh[2]), (k // mesh[2]) % mesh[1], k % mesh[2])
                    for k in range(nk)])
    m = np.array(mesh)

    def lin(v):
        v = np.mod(v, m)
        return (v[..., 0] * mesh[1] + v[..., 1]) * mesh[2] + v[..., 2]

    kmq = lin(vec[None, :, :] - vec[:, None, :])  # [Q, k]
    negq = lin(-vec)
    return kmq.astype(np.int64), negq.astype(np.int64)


def blocked(Gh, nk, nocc, m):
    """View Gh[w, (k1 a), (k2 r)] as Gb[w, k1, a, k2, r]."""
    return Gh.reshape(Gh.shape[0], nk, nocc, nk, m)


# ---------------------------------------------------------------------------
# one-time preparation
# ---------------------------------------------------------------------------

def half_rotate(L, A):
    """Half-rotated Cholesky vectors Lh[Q][k][a][r][g] = sum_p conj(A[k][p,a]) L[Q][k][p,r,g].

    k-point section: the half-transformed Cholesky matrix applies the trial's
    conjugated orbitals at k to the first band index.
    """
    nk = L.shape[0]
    Lh = np.empty((nk, nk, A.shape[2], L.shape[3], L.shape[4]), dtype=np.complex128)
    for Q in range(nk):
        for k in range(nk):
            Lh[Q, k] = np.tensordot(A[k].conj().T, L[Q, k], axes=(1, 0))
    return Lh


def h1_half(H1, A):
    """Half-rotated one-body blocks h1h[k] = A[k]^H H1[k] (nocc x m)."""
    return np.einsum("kpa,kpq->kaq", A.conj(), H1)


def mean_field_v0(L):
    """V0[k] = -1/2 sum_{Q,g} L[Q][k][:,:,g] L[Q][k][:,:,g]^H.

    Normal-ordering one-body term of the sum-of-squares two-body Hamiltonian
    (Introduction to AFQMC: v0 = -1/2 sum_r v_prrq), block diagonal in k.
    """
    nk, _, m, _, _ = L.shape
    V0 = np.zeros((nk, m, m), dtype=np.complex128)
    for k in range(nk):
        for Q in range(nk):
            blk = L[Q, k].reshape(m, -1)  # [p, (r g)]
            V0[k] -= 0.5 * blk @ blk.conj().T
    return V0


def one_body_propagator(H1, V0, dt):
    """Bhalf[k] = exp(-dt/2 (H1[k] + V0[k])) via the Hermitian eigendecomposition."""
    nk, m, _ = H1.shape
    B = np.empty_like(H1)
    for k in range(nk):
        hp = H1[k] + V0[k]
        hp = 0.5 * (hp + hp.conj().T)
        e, v = np.linalg.eigh(hp)
        B[k] = (v * np.exp(-0.5 * dt * e)) @ v.conj().T
    return B


def prepare(L, H1, A, dt):
    """All static data: Lh, h1h, V0 and Bhalf."""
    Lh = half_rotate(L, A)
    h1h = h1_half(H1, A)
    V0 = mean_field_v0(L)
    Bh = one_body_propagator(H1, V0, dt)
    return dict(Lh=Lh, h1h=h1h, V0=V0, bhalf=Bh)


# ---------------------------------------------------------------------------
# overlap and Green's function
# ---------------------------------------------------------------------------

def overlap_matrix(U, A):
    """O[w] = A^H U[w] with A block diagonal: O[(k a), j] = sum_p conj(A[k][p,a]) U[(k p), j]."""
    nw, N, nel = U.shape
    nk, m, nocc = A.shape
    Ub = U.reshape(nw, nk, m, nel)
    O = np.einsum("kpa,wkpj->wkaj", A.conj(), Ub).reshape(nw, nk * nocc, nel)
    return O


def greens(U, A):
    """Half-rotated Green's function and log overlap.

    Green's-function equations of the standard representation:
    Gh = (U^T A^*)^{-1} U^T = (O^T)^{-1} U^T with O = A^H U, computed with a
    linear solve.  logdet[w] = log det O[w] (complex); the closed-shell overlap
    is exp(2 logdet).
    """
    O = overlap_matrix(U, A)
    nw = U.shape[0]
    Gh = np.empty((nw, O.shape[1], U.shape[1]), dtype=np.complex128)
    logdet = np.empty(nw, dtype=np.complex128)
    for w in range(nw):
        sgn, la = np.linalg.slogdet(O[w])
        logdet[w] = la + 1j * np.angle(sgn)
        Gh[w] = np.linalg.solve(O[w].T, U[w].T)
    return Gh, logdet


# ---------------------------------------------------------------------------
# force bias
# ---------------------------------------------------------------------------

def cholesky_trace(Lh, Gh, mesh):
    """X[w][Q][g] = 2 sum_k sum_{a,r} Lh[Q][k][a,r,g] Gh[w][(k a), ((k-Q) r)].

    The trace of each (Q, g) potential against the Green's function, both spins
    (k-point force-bias equation).
    """
    nk, _, nocc, m, nchol = Lh.shape
    kmq, _ = kpoint_tables(mesh)
    Gb = blocked(Gh, nk, nocc, m)
    nw = Gh.shape[0]
    X = np.zeros((nw, nk, nchol), dtype=np.complex128)
    for Q in range(nk):
        for k in range(nk):
            g = Gb[:, k, :, kmq[Q, k], :]  # [w, a, r]
            X[:, Q, :] += np.tensordot(g, Lh[Q, k], axes=([1, 2], [0, 1]))
    return 2.0 * X


def force_bias(Lh, Gh, mesh, dt):
    """xbar[w][Q][g][+/-] and X (k-point force bias with (Q, -Q) symmetry).

    xbar+ = -sqrt(dt) (i/2) (X_Q + X_-Q),  xbar- = -sqrt(dt) (1/2) (X_Q - X_-Q).
    """
    _, negq = kpoint_tables(mesh)
    X = cholesky_trace(Lh, Gh, mesh)
    Xm = X[:, negq, :]
    sdt = np.sqrt(dt)
    xbar = np.empty(X.shape + (2,), dtype=np.complex128)
    xbar[..., 0] = -sdt * 0.5j * (X + Xm)
    xbar[..., 1] = -sdt * 0.5 * (X - Xm)
    return xbar, X


# ---------------------------------------------------------------------------
# HS potential
# ---------------------------------------------------------------------------

def combined_field(x, xbar, mesh):
    """zeta[w][Q][g] = -xi, xi = 1/2 [ i (xt+_Q + xt+_-Q) + (xt-_Q - xt-_-Q) ], xt = x - xbar."""
    _, negq = kpoint_tables(mesh)
    xt = x - xbar
    xp, xm = xt[..., 0], xt[..., 1]
    xi = 0.5 * (1j * (xp + xp[:, negq, :]) + (xm - xm[:, negq, :]))
    return -xi


def hs_potential(L, zeta, mesh):
    """vhs[w][(k p), ((k-Q) r)] = sum_g L[Q][k][p, r, g] zeta[w][Q][g] (dense per walker)."""
    nk, _, m, _, nchol = L.shape
    kmq, _ = kpoint_tables(mesh)
    nw = zeta.shape[0]
    vhs = np.zeros((nw, nk * m, nk * m), dtype=np.complex128)
    for Q in range(nk):
        for k in range(nk):
            k2 = kmq[Q, k]
            blk = np.tensordot(zeta[:, Q, :], L[Q, k], axes=(1, 2))  # [w, p, r]
            vhs[:, k * m:(k + 1) * m, k2 * m:(k2 + 1) * m] = blk
    return vhs


# ---------------------------------------------------------------------------
# propagation and weights
# ---------------------------------------------------------------------------

def apply_block_diag(B, U):
    """(blockdiag_k B[k]) @ U[w] for every walker."""
    nk, m, _ = B.shape
    nw, N, nel = U.shape
    Ub = U.reshape(nw, nk, m, nel)
    return np.einsum("kpq,wkqj->wkpj", B, Ub).reshape(nw, N, nel)


def taylor_exp_apply(V, U, order=6):
    """sum_{j=0..order} V^j U / j!, term by term: T_0 = U, T_j = V T_{j-1} / j."""
    acc = U.copy()
    term = U
    for j in range(1, order + 1):
        term = np.matmul(V, term) / j
        acc = acc + term
    return acc


def propagate(U, vhs, bhalf, dt, order=6):
    """U' = Bhalf T_order(-sqrt(dt) vhs) Bhalf U (symmetric Trotter walker propagator)."""
    T = apply_block_diag(bhalf, U)
    T = taylor_exp_apply(-np.sqrt(dt) * vhs, T, order)
    return apply_block_diag(bhalf, T)


def weight_update(logdet_old, logdet_new, x, xbar, w_old, shift=0.0):
    """Hybrid phaseless weight update.

    r = (det O'/det O)^2; I = r exp(sum (x xbar - xbar^2/2)) (bilinear, summed
    over Q, g and +/-); dtheta = arg r; w' = |I| max(0, cos dtheta) e^shift w, where
    shift = dt E_T is the energy shift of the projector exp(-dt (H - E_T)) (0: none).
    Returns (w_new, log_I, dtheta).
    """
    log_r = 2.0 * (logdet_new - logdet_old)
    s = np.sum(x * xbar - 0.5 * xbar * xbar, axis=(1, 2, 3))
    log_I = log_r + s
    dtheta = np.angle(np.exp(1j * log_r.imag))
    w_new = np.exp(log_I.real + shift) * np.maximum(0.0, np.cos(dtheta)) * w_old
    return w_new, log_I, dtheta


def orthonormalize(U):
    """Thin QR per walker, with the phases fixed so that diag(R) is real positive."""
    out = np.empty_like(U)
    for w in range(U.shape[0]):
        q, r = np.linalg.qr(U[w])
        d = np.diag(r)
        ph = d / np.abs(d)
        out[w] = q * ph[None, :]
    return out


def step(U, logdet, weight, x, pre, A, L, mesh, dt, order=6, etrial=0.0):
    """One walker-batch step: force bias -> HS potential -> propagate -> G, weights (with
    the energy shift E_T = etrial per supercell)."""
    Gh, _ = greens(U, A)
    xbar, X = force_bias(pre["Lh"], Gh, mesh, dt)
    zeta = combined_field(x, xbar, mesh)
    vhs = hs_potential(L, zeta, mesh)
    U2 = propagate(U, vhs, pre["bhalf"], dt, order)
    Gh2, logdet2 = greens(U2, A)
    w2, log_I, dth = weight_update(logdet, logdet2, x, xbar, weight, shift=dt * etrial)
    return dict(U=U2, Gh=Gh2, logdet=logdet2, weight=w2, xbar=xbar, X=X, vhs=vhs,
                log_I=log_I, dtheta=dth)


# ---------------------------------------------------------------------------
# local energy (paper's energy-evaluation algorithm, steps 1-3)
# ---------------------------------------------------------------------------

def local_energy(Lh, h1h, Gh, mesh, walkers=None):
    """E[w] = (E1B, EC, EX) per supercell, complex128.

    Step 1: reshape Gh[w, (k1 a), (k2 q)] -> G[k1, k2, w, a, q].
    Step 2: for each (Q, k, k'):
      T1[w,b,a,g] = sum_r Lh[Q][k][a,r,g]      G[k'-Q, k-Q, w, b, r]
      T2[w,a,b,g] = sum_s Lh[-Q][k'-Q][b,s,g]  G[k, k', w, a, s]
      EX[w] += -(1/2) * 2 spins * sum_{a,b,g} T1[w,b,a,g] T2[w,a,b,g]
      when k' - Q = k: v1 += sum_a T1[w,a,a,g], v2 += sum_a T2[w,a,a,g]
    Step 3: EC = 1/2 sum_g (2 v1)(2 v2)  (both spins in each factor).
    One-body: E1B = 2 sum_k sum_{a,r} h1h[k][a,r] G[k, k, w, a, r].
    """
    nk, _, nocc, m, nchol = Lh.shape
    kmq, negq = kpoint_tables(mesh)
    if walkers is not None:
        Gh = Gh[walkers]
    nw = Gh.shape[0]
    G = np.ascontiguousarray(blocked(Gh, nk, nocc, m).transpose(1, 3, 0, 2, 4))
    EX = np.zeros(nw, dtype=np.complex128)
    v1 = np.zeros((nw, nk, nchol), dtype=np.complex128)
    v2 = np.zeros((nw, nk, nchol), dtype=np.complex128)
    for Q in range(nk):
        mQ = negq[Q]
        for k in range(nk):
            kq = kmq[Q, k]
            LA = Lh[Q, k]  # [a, r, g]
            for kp in range(nk):
                kpq = kmq[Q, kp]
                # T1[w, b, a, g]
                T1 = np.einsum("arg,wbr->wbag", LA, G[kpq, kq], optimize=True)
                # T2[w, a, b, g]
                T2 = np.einsum("bsg,was->wabg", Lh[mQ, kpq], G[k, kp], optimize=True)
                EX -= np.einsum("wbag,wabg->w", T1, T2, optimize=True)
                if kpq == k:
                    v1[:, Q, :] += np.einsum("waag->wg", T1)
                    v2[:, Q, :] += np.einsum("waag->wg", T2)
    EC = 0.5 * np.sum((2.0 * v1) * (2.0 * v2), axis=(1, 2))
    E1 = np.zeros(nw, dtype=np.complex128)
    for k in range(nk):
        E1 += 2.0 * np.einsum("ar,war->w", h1h[k], G[k, k])
    return np.stack([E1, EC, EX], axis=1)


def mixed_energy(E_parts, weight):
    """Mixed estimate of the energy (the mixed-estimate equation of the standard-
    representation section): sum_a w_a E_L[phi_a] / sum_a w_a, with E_L the sum of the
    three parts (one-body, Coulomb, exchange) per walker."""
    EL = np.asarray(E_parts).sum(axis=1)
    w = np.asarray(weight, dtype=float)
    return complex((w * EL).sum() / w.sum())


def energy_gradient(Lh, h1h, Gh, mesh, walkers=None):
    """dE/dGh[w][(k1 al), (k2 rho)] of the local energy above (holomorphic derivative).

    E is a quadratic polynomial in Gh without conjugates, so the derivative is
    the ordinary complex one:
      2 [ h1h[k1][al,rho] delta(k1,k2)
        + sum_g Lh[Q0][k1][al,rho,g] X[-Q0][g],               Q0 = k1 - k2
        - sum_{Q,g,b,r} Lh[Q][k1][al,r,g] Lh[-Q][k2-Q][b,rho,g] G[(k2-Q) b, (k1-Q) r] ]
    The exchange part recomputes T1 of the energy algorithm for (Q, k1, k2) and
    contracts it with Lh[-Q][k2-Q] over (b, g); the two G factors of the
    exchange term contribute equally.
    """
    nk, _, nocc, m, nchol = Lh.shape
    kmq, negq = kpoint_tables(mesh)
    if walkers is not None:
        Gh = Gh[walkers]
    nw = Gh.shape[0]
    X = cholesky_trace(Lh, Gh, mesh)
    G = np.ascontiguousarray(blocked(Gh, nk, nocc, m).transpose(1, 3, 0, 2, 4))
    D = np.zeros((nw, nk, nocc, nk, m), dtype=np.complex128)
    # qidx[k1, k2] = k1 - k2
    qidx = np.empty((nk, nk), dtype=np.int64)
    for Q in range(nk):
        for k in range(nk):
            qidx[k, kmq[Q, k]] = Q
    for k1 in range(nk):
        D[:, k1, :, k1, :] += h1h[k1][None]
        for k2 in range(nk):
            Q0 = qidx[k1, k2]
            D[:, k1, :, k2, :] += np.einsum("arg,wg->war", Lh[Q0, k1], X[:, negq[Q0], :])
            for Q in range(nk):
                T1 = np.einsum("arg,wbr->wbag", Lh[Q, k1], G[kmq[Q, k2], kmq[Q, k1]],
                               optimize=True)
                D[:, k1, :, k2, :] -= np.einsum("wbag,bsg->was", T1,
                                                Lh[negq[Q], kmq[Q, k2]], optimize=True)
    return 2.0 * D.reshape(nw, nk * nocc, nk * m)
