"""Collinear spin-unrestricted walkers in the k-point representation, FP64 (test
infrastructure only: imported by tests, the repository smoke check and the benchmark's
CPU-baseline leg, never by the GPU library; it shares no code with it).

The Hamiltonian of "Introduction to AFQMC" sums over the spins sigma, sigma' of the two
electrons; the closed-shell walker stores one determinant for both.  A collinear walker
(an unrestricted, UHF-type determinant) keeps one determinant per spin, U_up
(nk m x nk n_up) and U_dn (nk m x nk n_dn), against a trial with one block-diagonal
determinant per spin, A_up[k] (m x n_up) and A_dn[k] (m x n_dn).  The single-particle
basis is the same for both spins ("k-Point Representation": spin-independent h and L), so:

* half rotation per spin: Lh^s[Q][k][a][r][g] = sum_p conj(A_s[k][p,a]) L[Q][k][p,r,g],
  h1h^s[k] = A_s[k]^H H1[k];
* force bias: X[Q][g] = sum_s sum_k sum_{a,r} Lh^s[Q][k][a,r,g] Gh^s[(k a), ((k-Q) r)], the
  trace over both spins, and xbar from X exactly as for the closed shell (where the two
  spin traces are equal, X = 2 x one);
* propagation: both spins' determinants take the same one- and two-body operators (one
  field per walker);
* overlap: <Psi_T|phi> = det(A_up^H U_up) det(A_dn^H U_dn), so the weight update takes the
  sum of the two spins' log-overlap changes where the closed shell takes twice one;
* local energy, the energy-evaluation steps with their loop over sigma:
    E1 = sum_s sum_k sum_{a,r} h1h^s[k][a,r] G^s[k,k][a,r]
    T1^s[b,a,g] = sum_r Lh^s[Q][k][a,r,g] G^s[k'-Q, k-Q][b,r]
    T2^s[a,b,g] = sum_s' Lh^s[-Q][k'-Q][b,s',g] G^s[k, k'][a,s']
    EX = -1/2 sum_s sum_{Q,k,k'} sum_{a,b,g} T1^s T2^s
    v1, v2 += the diagonal traces of T1^s, T2^s for k'-Q = k (over both spins)
    EC = 1/2 sum_{Q,g} v1 v2;
* adjoint: dE/dGh^s[(k1 al), (k2 rho)] = h1h^s[k1][al,rho] delta(k1,k2)
    + sum_g Lh^s[Q0][k1][al,rho,g] X[-Q0][g]  (Q0 = k1 - k2)
    - sum_{Q,g,b,r} Lh^s[Q][k1][al,r,g] Lh^s[-Q][k2-Q][b,rho,g] G^s[(k2-Q) b, (k1-Q) r].

Pinned by tests/test_oracle_pins.py: equal spins reproduce the closed-shell oracle (energy,
force bias, gradient halves, step and weights); the energy equals the generic
spin-resolved expression with explicit 4-index integrals of the supercell; it is invariant
under swapping the spins; the gradient matches finite differences; the overlap ratio of a
step matches dense determinants of the supercell.
"""

from __future__ import annotations

import numpy as np

from . import kpoint as kp


def prepare(L, H1, A_up, A_dn, dt):
    """Per-spin half rotations and the shared one-body propagator."""
    V0 = kp.mean_field_v0(L)
    return dict(Lh=(kp.half_rotate(L, A_up), kp.half_rotate(L, A_dn)),
                h1h=(kp.h1_half(H1, A_up), kp.h1_half(H1, A_dn)),
                V0=V0, bhalf=kp.one_body_propagator(H1, V0, dt))


def _trace(Lh, Gh, mesh):
    """sum_k sum_{a,r} Lh[Q][k][a,r,g] Gh[w][(k a), ((k-Q) r)] for one spin."""
    nk, _, n, m, nchol = Lh.shape
    kmq, _ = kp.kpoint_tables(mesh)
    Gb = kp.blocked(Gh, nk, n, m)
    X = np.zeros((Gh.shape[0], nk, nchol), dtype=np.complex128)
    for Q in range(nk):
        for k in range(nk):
            X[:, Q, :] += np.tensordot(Gb[:, k, :, kmq[Q, k], :], Lh[Q, k], axes=([1, 2], [0, 1]))
    return X


def cholesky_trace(Lh, Gh, mesh):
    """X[w][Q][g], summed over the two spins (Lh, Gh: pairs (up, down))."""
    return _trace(Lh[0], Gh[0], mesh) + _trace(Lh[1], Gh[1], mesh)


def force_bias(Lh, Gh, mesh, dt):
    """xbar[w][Q][g][+/-] from the two-spin trace X, and X."""
    _, negq = kp.kpoint_tables(mesh)
    X = cholesky_trace(Lh, Gh, mesh)
    Xm = X[:, negq, :]
    sdt = np.sqrt(dt)
    xbar = np.empty(X.shape + (2,), dtype=np.complex128)
    xbar[..., 0] = -sdt * 0.5j * (X + Xm)
    xbar[..., 1] = -sdt * 0.5 * (X - Xm)
    return xbar, X


def local_energy(Lh, h1h, Gh, mesh):
    """E[w] = (E1B, EC, EX) per supercell of the two-determinant walkers."""
    nk, _, _, m, nchol = Lh[0].shape
    kmq, negq = kp.kpoint_tables(mesh)
    nw = Gh[0].shape[0]
    E1 = np.zeros(nw, dtype=np.complex128)
    EX = np.zeros(nw, dtype=np.complex128)
    v1 = np.zeros((nw, nk, nchol), dtype=np.complex128)
    v2 = np.zeros((nw, nk, nchol), dtype=np.complex128)
    for s in range(2):
        n = Lh[s].shape[2]
        # step 1: G^s[k1, k2, w, a, q]
        G = np.ascontiguousarray(kp.blocked(Gh[s], nk, n, m).transpose(1, 3, 0, 2, 4))
        for Q in range(nk):
            mQ = negq[Q]
            for k in range(nk):
                kq = kmq[Q, k]
                for kpt in range(nk):
                    kpq = kmq[Q, kpt]
                    T1 = np.einsum("arg,wbr->wbag", Lh[s][Q, k], G[kpq, kq], optimize=True)
                    T2 = np.einsum("bsg,was->wabg", Lh[s][mQ, kpq], G[k, kpt], optimize=True)
                    EX -= 0.5 * np.einsum("wbag,wabg->w", T1, T2, optimize=True)
                    if kpq == k:
                        v1[:, Q, :] += np.einsum("waag->wg", T1)
                        v2[:, Q, :] += np.einsum("waag->wg", T2)
        for k in range(nk):
            E1 += np.einsum("ar,war->w", h1h[s][k], G[k, k])
    EC = 0.5 * np.sum(v1 * v2, axis=(1, 2))
    return np.stack([E1, EC, EX], axis=1)


def energy_gradient(Lh, h1h, Gh, mesh):
    """(dE/dGh^up, dE/dGh^dn) of the local energy above (holomorphic derivatives)."""
    nk, _, _, m, _ = Lh[0].shape
    kmq, negq = kp.kpoint_tables(mesh)
    nw = Gh[0].shape[0]
    X = cholesky_trace(Lh, Gh, mesh)
    qidx = np.empty((nk, nk), dtype=np.int64)  # qidx[k1, k2] = k1 - k2
    for Q in range(nk):
        for k in range(nk):
            qidx[k, kmq[Q, k]] = Q
    out = []
    for s in range(2):
        n = Lh[s].shape[2]
        G = np.ascontiguousarray(kp.blocked(Gh[s], nk, n, m).transpose(1, 3, 0, 2, 4))
        D = np.zeros((nw, nk, n, nk, m), dtype=np.complex128)
        for k1 in range(nk):
            D[:, k1, :, k1, :] += h1h[s][k1][None]
            for k2 in range(nk):
                Q0 = qidx[k1, k2]
                D[:, k1, :, k2, :] += np.einsum("arg,wg->war", Lh[s][Q0, k1], X[:, negq[Q0], :])
                for Q in range(nk):
                    T1 = np.einsum("arg,wbr->wbag", Lh[s][Q, k1], G[kmq[Q, k2], kmq[Q, k1]],
                                   optimize=True)
                    D[:, k1, :, k2, :] -= np.einsum("wbag,bsg->was", T1,
                                                    Lh[s][negq[Q], kmq[Q, k2]], optimize=True)
        out.append(D.reshape(nw, nk * n, nk * m))
    return tuple(out)


def weight_update(logdet_old, logdet_new, x, xbar, w_old, shift=0.0):
    """Hybrid phaseless weight update with the two-determinant overlap:
    r = prod_s det O'_s / det O_s; I = r exp(sum (x xbar - xbar^2/2)); dtheta = arg r;
    w' = |I| max(0, cos dtheta) e^shift w.  logdet_*: pairs (up, down)."""
    log_r = (logdet_new[0] - logdet_old[0]) + (logdet_new[1] - logdet_old[1])
    s = np.sum(x * xbar - 0.5 * xbar * xbar, axis=(1, 2, 3))
    log_I = log_r + s
    dtheta = np.angle(np.exp(1j * log_r.imag))
    w_new = np.exp(log_I.real + shift) * np.maximum(0.0, np.cos(dtheta)) * w_old
    return w_new, log_I, dtheta


def step(U, logdet, weight, x, pre, A, L, mesh, dt, order=6, etrial=0.0):
    """One step of two-determinant walkers: U, logdet, A pairs (up, down); one field x per
    walker for both spins."""
    Gh = tuple(kp.greens(U[s], A[s])[0] for s in range(2))
    xbar, X = force_bias(pre["Lh"], Gh, mesh, dt)
    zeta = kp.combined_field(x, xbar, mesh)
    vhs = kp.hs_potential(L, zeta, mesh)
    U2 = tuple(kp.propagate(U[s], vhs, pre["bhalf"], dt, order) for s in range(2))
    g2 = [kp.greens(U2[s], A[s]) for s in range(2)]
    Gh2 = (g2[0][0], g2[1][0])
    ld2 = (g2[0][1], g2[1][1])
    w2, log_I, dth = weight_update(logdet, ld2, x, xbar, weight, shift=dt * etrial)
    return dict(U=U2, Gh=Gh2, logdet=ld2, weight=w2, xbar=xbar, X=X, vhs=vhs,
                log_I=log_I, dtheta=dth)
