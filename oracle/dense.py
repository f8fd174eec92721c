"""The standard (dense) representation of a k-point system, FP64 (test infrastructure only:
imported by tests, the repository smoke check and the benchmark's CPU-baseline leg, never by
the GPU library; it shares no code with it).

The standard representation of the paper works with one set of Cholesky vectors of the whole
supercell basis (M = Nk m orbitals).  Its HS construction with one real field per vector
needs Hermitian vectors.  The supercell operators of the k-point factorisation are Hermitian
only for Q = -Q; otherwise the pair (Q, -Q) carries LL_Q and LL_{-Q} = LL_Q^H, and the two
Hermitian combinations
    A = (LL_Q + LL_Q^H) / sqrt 2,      B = i (LL_Q - LL_Q^H) / sqrt 2
reproduce the pair's part of the integrals, A (x) A^H + B (x) B^H = LL_Q (x) LL_Q^H +
LL_{-Q} (x) LL_{-Q}^H, and of V0, A A^H + B B^H = LL_Q LL_Q^H + LL_{-Q} LL_{-Q}^H.  So the
dense set has Nk C Hermitian vectors: for every Q with index <= that of -Q, in increasing Q,
the C vectors LL_Q (Q = -Q) or the 2C vectors A_0 .. A_{C-1}, B_0 .. B_{C-1}.

Fields.  The k-point HS exponent takes per pair (Q, -Q) and Cholesky index g the combination
xi_Q LL_Q + xi_{-Q} LL_Q^H (xi of the field combination), the dense one i x_A A + i x_B B.
They are equal for x_A = (x+_Q + x+_{-Q}) / sqrt 2 and x_B = (x-_{-Q} - x-_Q) / sqrt 2, an
orthogonal change of the Gaussian fields whose other two directions do not enter the
exponent and carry no force bias; for Q = -Q, x = x+_Q.  The dense minus fields are unused
(a Hermitian vector has no minus potential) and set to zero.

Pinned by tests/test_oracle_pins.py: the dense vectors are Hermitian, give the explicit
4-index integrals and V0 of the unfolded k-point operators, the dense energy equals the
k-point energy, and one step with the mapped fields equals the k-point step.
"""

from __future__ import annotations

import numpy as np

from . import kpoint as kp
from . import supercell as sc


def dense_slots(mesh):
    """The Q with index <= that of -Q, increasing, and whether each is its own partner."""
    _, negq = kp.kpoint_tables(mesh)
    return [(Q, Q == negq[Q]) for Q in range(len(negq)) if Q <= negq[Q]]


def dense_cholesky(L, mesh):
    """Hermitian dense vectors as L_d[0][0][P][R][gd] (the library's layout for a 1x1x1
    mesh), gd over the slots of dense_slots."""
    nk, _, m, _, C = L.shape
    LL = sc.unfold_cholesky(L, mesh).reshape(nk, C, nk * m, nk * m)
    vecs = []
    for Q, self_paired in dense_slots(mesh):
        if self_paired:
            vecs.append(LL[Q])
        else:
            LH = LL[Q].conj().transpose(0, 2, 1)
            vecs.append((LL[Q] + LH) / np.sqrt(2.0))
            vecs.append(1j * (LL[Q] - LH) / np.sqrt(2.0))
    D = np.concatenate(vecs, axis=0)  # [gd, P, R]
    return np.ascontiguousarray(D.transpose(1, 2, 0))[None, None]


def dense_one_body(H1, A):
    """H1_d[0] = blockdiag(H1[k]), A_d[0] = blockdiag(A[k])."""
    return sc.block_diag(H1)[None], sc.block_diag(A)[None]


def dense_fields(x, mesh):
    """Dense fields [W][1][Nk C][2] from k-point fields x[W][Q][C][+/-]."""
    _, negq = kp.kpoint_tables(mesh)
    W, nk, C, _ = x.shape
    out = []
    for Q, self_paired in dense_slots(mesh):
        if self_paired:
            out.append(x[:, Q, :, 0])
        else:
            mQ = negq[Q]
            out.append((x[:, Q, :, 0] + x[:, mQ, :, 0]) / np.sqrt(2.0))
            out.append((x[:, mQ, :, 1] - x[:, Q, :, 1]) / np.sqrt(2.0))
    xp = np.concatenate(out, axis=1)  # [W, nk C]
    xd = np.zeros((W, 1, nk * C, 2))
    xd[:, 0, :, 0] = xp
    return xd
