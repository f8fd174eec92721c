"""Non-uniform band counts per k-point, FP64 (test infrastructure only: imported by tests,
the repository smoke check and the benchmark's CPU-baseline leg, never by the GPU library;
it shares no code with it).

The k-point representation counts an average of m bands per k-point: the basis at k may
hold mk[k] bands, so the block (Q, k) of the Cholesky vectors is mk[k] x mk[k-Q] and the
one-body block at k is mk[k] x mk[k].  Two routes to such a system:

* supercell: the dense operators of the M = sum_k mk[k] orbital basis (blocks placed at
  the band offsets of their k-points), for the generic expressions of the standard
  representation (supercell module);
* padding: every k-point padded to m >= max mk bands with zero rows and columns in L, H1
  and the trial, and zero rows in the walkers.  The padded bands carry no one-body or
  two-body matrix element, so each walker's padded rows stay zero under the propagator
  (the padded block of exp(-dt/2 (H1 + V0)) is the identity, that of the HS potential
  zero), the overlap A^H U and the Green's function ignore them, and every trace and
  contraction of the method is unchanged: the padded uniform system is the same system.

Pinned by tests/test_oracle_pins.py: the padded system's k-point energy, force bias and
step equal the supercell route's for the ragged system.
"""

from __future__ import annotations

import numpy as np

from . import kpoint as kp


def offsets(mk):
    """Band offset of each k-point in the supercell basis, and the total M."""
    o = np.concatenate([[0], np.cumsum(mk)]).astype(np.int64)
    return o[:-1], int(o[-1])


def supercell(rs):
    """(LL[(Q g), P, R], h, Af) of the ragged system: block (k, k - Q) of (Q, g) is
    L[Q][k][:, :, g]; h and Af block diagonal over k."""
    nk, C = rs.nk, rs.nchol
    kmq, _ = kp.kpoint_tables(rs.mesh)
    off, M = offsets(rs.mk)
    LL = np.zeros((nk, C, M, M), dtype=np.complex128)
    for Q in range(nk):
        for k in range(nk):
            k2 = kmq[Q, k]
            LL[Q, :, off[k]:off[k] + rs.mk[k], off[k2]:off[k2] + rs.mk[k2]] = \
                rs.L[Q][k].transpose(2, 0, 1)
    h = np.zeros((M, M), dtype=np.complex128)
    Af = np.zeros((M, nk * rs.nocc), dtype=np.complex128)
    for k in range(nk):
        h[off[k]:off[k] + rs.mk[k], off[k]:off[k] + rs.mk[k]] = rs.H1[k]
        Af[off[k]:off[k] + rs.mk[k], k * rs.nocc:(k + 1) * rs.nocc] = rs.A[k]
    return LL.reshape(nk * C, M, M), h, Af


def pad(rs, m):
    """Uniform arrays with m bands per k-point: L [nk][nk][m][m][nchol], H1 [nk][m][m],
    A [nk][m][nocc], zero beyond each k-point's own bands."""
    nk, C = rs.nk, rs.nchol
    kmq, _ = kp.kpoint_tables(rs.mesh)
    L = np.zeros((nk, nk, m, m, C), dtype=np.complex128)
    H1 = np.zeros((nk, m, m), dtype=np.complex128)
    A = np.zeros((nk, m, rs.nocc), dtype=np.complex128)
    for Q in range(nk):
        for k in range(nk):
            L[Q, k, :rs.mk[k], :rs.mk[kmq[Q, k]]] = rs.L[Q][k]
    for k in range(nk):
        H1[k, :rs.mk[k], :rs.mk[k]] = rs.H1[k]
        A[k, :rs.mk[k]] = rs.A[k]
    return L, H1, A


def pad_walkers(U, mk, m):
    """Rows of ragged walkers [W][sum mk][n] to the padded [W][nk m][n]."""
    off, _ = offsets(mk)
    W, _, n = U.shape
    out = np.zeros((W, len(mk) * m, n), dtype=U.dtype)
    for k, mq in enumerate(mk):
        out[:, k * m:k * m + mq] = U[:, off[k]:off[k] + mq]
    return out


def unpad_walkers(U, mk, m):
    """Padded walkers [W][nk m][n] back to the ragged rows [W][sum mk][n]."""
    off, M = offsets(mk)
    out = np.empty((U.shape[0], M, U.shape[2]), dtype=U.dtype)
    for k, mq in enumerate(mk):
        out[:, off[k]:off[k] + mq] = U[:, k * m:k * m + mq]
    return out


def unpad_greens(Gh, mk, m):
    """Padded half-rotated Green's functions [W][n][nk m] to the ragged columns
    [W][n][sum mk]."""
    off, M = offsets(mk)
    out = np.empty((Gh.shape[0], Gh.shape[1], M), dtype=Gh.dtype)
    for k, mq in enumerate(mk):
        out[:, :, off[k]:off[k] + mq] = Gh[:, :, k * m:k * m + mq]
    return out
