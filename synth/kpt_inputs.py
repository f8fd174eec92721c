"""Seeded generator for k-point AFQMC inputs.

Shapes follow the momentum-blocked statement of the problem (Sec. "k-Point
Representation"): the one-body Hamiltonian is block diagonal in k, and the
Cholesky vectors carry a momentum transfer Q with the second band index at
k - Q.  Sizes mirror carbon in the diamond structure with a GTH-DZVP basis
(13 functions per atom, two atoms per cell, 8 valence electrons per cell,
Sec. "Scaling and Performance").

Everything is drawn from one numpy PCG64 stream, in this order:

1. H1[k] for k = 0..nk-1: diag(linspace(-1, 2, m)) plus the off-diagonal part
   of (C + C^H)/2, with C = 0.05 * CN(0, 1) of shape (m, m).
2. L[Q][k] for Q = 0..nk-1, k = 0..nk-1, when the block is still unset:
   Z = CN(0, 1) of shape (m, m, nchol), scaled per vector by exp(-g/6)/sqrt(m).
   The time-reversal partner (-Q, k-Q) is filled with the conjugate transpose
   in (i, l) (the (Q, -Q) relation of the k-point section); when the partner is
   the block itself (Q = 0) the block is made Hermitian in (i, l).
3. Trial orbitals A[k] (m x nocc): the first nocc identity columns, or, with
   trial="random", the Q factor of a complex Gaussian (m x nocc) matrix.
4. Walkers (make_walkers): block diagonal, blockdiag_k QR(A[k] + 0.1 CN(0,1)),
   or dense, QR of a CN(0,1) (nk*m x nk*nocc) matrix.
5. Fields (make_fields): x ~ N(0, 1) of shape (nsteps, nwalk, nk, nchol, 2),
   the last axis being the (+, -) potentials.

CN(0, 1) = (N(0,1) + i N(0,1)) / sqrt(2); the real parts of a block are drawn
before its imaginary parts.  k is linearised row-major over the mesh,
k = (k0 * mesh1 + k1) * mesh2 + k2, and k - Q, -Q are componentwise mod mesh.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# The five workloads (nk from the mesh; nchol = 8 m unless stated).
CONFIGS = {
    "c0": dict(mesh=(2, 2, 2), m=8, nocc=2, nchol=24, nwalk=4, nsteps=1, seed=0),
    "c1": dict(mesh=(3, 3, 3), m=26, nocc=4, nchol=208, nwalk=64, nsteps=20, seed=0),
    "c2": dict(mesh=(4, 4, 4), m=52, nocc=4, nchol=400, nwalk=32, nsteps=10, seed=0),
    "c3A": dict(mesh=(2, 2, 2), m=26, nocc=4, nchol=208, nwalk=128, nsteps=10, seed=1),
    "c3B": dict(mesh=(3, 3, 3), m=26, nocc=4, nchol=208, nwalk=64, nsteps=10, seed=2),
    "c3C": dict(mesh=(3, 3, 3), m=52, nocc=4, nchol=416, nwalk=32, nsteps=10, seed=3),
    "c4": dict(mesh=(3, 3, 3), m=26, nocc=4, nchol=208, nwalk=16, nsteps=0, seed=0),
}

DT = 0.005


def config_shapes(name: str) -> dict:
    """Return a copy of the shape dictionary of a named workload."""
    c = dict(CONFIGS[name])
    c["nk"] = int(np.prod(c["mesh"]))
    c["dt"] = DT
    return c


@dataclass
class KptSystem:
    mesh: tuple
    m: int
    nocc: int
    nchol: int
    dt: float
    H1: np.ndarray  # [nk, m, m] complex128, Hermitian blocks
    L: np.ndarray  # [nk(Q), nk(k), m(i at k), m(l at k-Q), nchol] complex128
    A: np.ndarray  # [nk, m, nocc] complex128, orthonormal columns
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def nk(self) -> int:
        return int(np.prod(self.mesh))


def _cn(rng: np.random.Generator, shape) -> np.ndarray:
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def _kvec(k: int, mesh) -> tuple:
    return (k // (mesh[1] * mesh[2]), (k // mesh[2]) % mesh[1], k % mesh[2])


def _klin(v, mesh) -> int:
    return ((v[0] % mesh[0]) * mesh[1] + (v[1] % mesh[1])) * mesh[2] + (v[2] % mesh[2])


def _partner(Q: int, k: int, mesh) -> tuple:
    """Block index (-Q, k-Q) that holds the conjugate transpose of block (Q, k)."""
    q = _kvec(Q, mesh)
    kv = _kvec(k, mesh)
    mq = _klin(tuple(-c for c in q), mesh)
    kmq = _klin(tuple(a - b for a, b in zip(kv, q)), mesh)
    return mq, kmq


def _cholesky_blocks(rng, mesh, m, nchol):
    """Yield (Q, k, L[Q][k]) in draw order: each block is drawn together with its
    time-reversal partner (-Q, k-Q), which follows it."""
    nk = int(np.prod(mesh))
    done = np.zeros((nk, nk), dtype=bool)
    scale = np.exp(-np.arange(nchol) / 6.0) / np.sqrt(m)
    for Q in range(nk):
        for k in range(nk):
            if done[Q, k]:
                continue
            z = _cn(rng, (m, m, nchol))
            pQ, pk = _partner(Q, k, mesh)
            if (pQ, pk) == (Q, k):
                blk = 0.5 * (z + z.conj().transpose(1, 0, 2))
                done[Q, k] = True
                yield Q, k, blk * scale
            else:
                blk = z * scale
                done[Q, k] = True
                done[pQ, pk] = True
                yield Q, k, blk
                yield pQ, pk, blk.conj().transpose(1, 0, 2)


def make_system(mesh, m, nocc, nchol, seed=0, dt=DT, trial="identity",
                rng: np.random.Generator | None = None,
                ldtype=np.complex128, sink=None) -> tuple[KptSystem, np.random.Generator]:
    """Draw H1, L and the trial; return the system and the still-live generator.

    With sink, L is not kept: sink(Q, k, block) receives each (m, m, nchol) block in draw
    order (for workloads whose L exceeds host memory) and the system's L is None.
    """
    mesh = tuple(int(v) for v in mesh)
    nk = int(np.prod(mesh))
    if nocc > m:
        raise ValueError("nocc must not exceed m")
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))

    H1 = np.empty((nk, m, m), dtype=np.complex128)
    base = np.diag(np.linspace(-1.0, 2.0, m))
    for k in range(nk):
        c = 0.05 * _cn(rng, (m, m))
        h = 0.5 * (c + c.conj().T)
        np.fill_diagonal(h, 0.0)
        H1[k] = base + h

    if sink is None:
        L = np.zeros((nk, nk, m, m, nchol), dtype=ldtype)

        def store(Q, k, blk):
            L[Q, k] = blk
    else:
        L = None
        store = sink
    for Q, k, blk in _cholesky_blocks(rng, mesh, m, nchol):
        store(Q, k, blk)

    if trial == "identity":
        A = np.zeros((nk, m, nocc), dtype=np.complex128)
        for k in range(nk):
            A[k, :nocc, :nocc] = np.eye(nocc)
    elif trial == "random":
        A = np.empty((nk, m, nocc), dtype=np.complex128)
        for k in range(nk):
            q, _ = np.linalg.qr(_cn(rng, (m, nocc)))
            A[k] = q
    else:
        raise ValueError(f"unknown trial kind {trial!r}")

    sysobj = KptSystem(mesh=mesh, m=m, nocc=nocc, nchol=nchol, dt=dt,
                       H1=H1, L=L, A=A, seed=seed)
    return sysobj, rng


def make_walkers(sysobj: KptSystem, nwalk: int, rng: np.random.Generator,
                 kind: str = "blockdiag", noise: float = 0.1) -> np.ndarray:
    """Walker orbitals U[w] of shape (nk*m, nk*nocc), complex128."""
    nk, m, nocc = sysobj.nk, sysobj.m, sysobj.nocc
    U = np.zeros((nwalk, nk * m, nk * nocc), dtype=np.complex128)
    for w in range(nwalk):
        if kind == "blockdiag":
            for k in range(nk):
                q, _ = np.linalg.qr(sysobj.A[k] + noise * _cn(rng, (m, nocc)))
                U[w, k * m:(k + 1) * m, k * nocc:(k + 1) * nocc] = q
        elif kind == "dense":
            q, _ = np.linalg.qr(_cn(rng, (nk * m, nk * nocc)))
            U[w] = q
        else:
            raise ValueError(f"unknown walker kind {kind!r}")
    return U


def make_fields(sysobj: KptSystem, nwalk: int, nsteps: int,
                rng: np.random.Generator) -> np.ndarray:
    """Auxiliary fields x[step, w, Q, g, +/-] ~ N(0, 1), float64."""
    return rng.standard_normal((nsteps, nwalk, sysobj.nk, sysobj.nchol, 2))


def make_config(name: str, walkers: str = "blockdiag", trial: str = "identity"):
    """System, walkers and fields of a named workload, drawn in generator order."""
    c = config_shapes(name)
    s, rng = make_system(c["mesh"], c["m"], c["nocc"], c["nchol"], seed=c["seed"],
                         dt=c["dt"], trial=trial)
    U = make_walkers(s, c["nwalk"], rng, kind=walkers)
    x = make_fields(s, c["nwalk"], max(c["nsteps"], 1), rng)
    return s, U, x


def make_spin_trial(sysobj: KptSystem, n_dn: int, rng: np.random.Generator,
                    mix: float = 0.3) -> np.ndarray:
    """Down-spin trial orbitals A_dn[k] (m x n_dn) of a collinear spin-polarised trial whose
    up-spin orbitals are sysobj.A: per k, the Q factor of the first min(n_dn, nocc) up-spin
    columns (zero columns beyond) plus mix * CN(0, 1) of shape (m, n_dn)."""
    nk, m, nocc = sysobj.nk, sysobj.m, sysobj.nocc
    if n_dn > m:
        raise ValueError("n_dn must not exceed m")
    A = np.empty((nk, m, n_dn), dtype=np.complex128)
    c = min(n_dn, nocc)
    for k in range(nk):
        B = np.zeros((m, n_dn), dtype=np.complex128)
        B[:, :c] = sysobj.A[k][:, :c]
        q, _ = np.linalg.qr(B + mix * _cn(rng, (m, n_dn)))
        A[k] = q
    return A


def spin_view(sysobj: KptSystem, A_spin: np.ndarray) -> KptSystem:
    """The same system with another spin's trial orbitals (for make_walkers)."""
    return KptSystem(mesh=sysobj.mesh, m=sysobj.m, nocc=A_spin.shape[2], nchol=sysobj.nchol,
                     dt=sysobj.dt, H1=sysobj.H1, L=sysobj.L, A=A_spin, seed=sysobj.seed,
                     extra=sysobj.extra)


@dataclass
class RaggedSystem:
    """A k-point system with mk[k] bands at k (non-uniform band counts).

    H1[k]: (mk[k], mk[k]); L[Q][k]: (mk[k], mk[k-Q], nchol); A[k]: (mk[k], nocc)."""
    mesh: tuple
    mk: tuple
    nocc: int
    nchol: int
    dt: float
    H1: list
    L: list
    A: list
    seed: int = 0

    @property
    def nk(self) -> int:
        return int(np.prod(self.mesh))


def make_ragged_system(mesh, mk, nocc, nchol, seed=0, dt=DT,
                       rng: np.random.Generator | None = None):
    """The generator of make_system with mk[k] bands at k: H1[k] diag(linspace(-1, 2,
    mk[k])) plus the off-diagonal part of (C + C^H)/2; L blocks of shape
    (mk[k], mk[k-Q], nchol) drawn with their time-reversal partners as in make_system
    (scale exp(-g/6)/sqrt(max mk)); random trial orbitals (Q factor of CN(0,1) (mk[k], nocc))."""
    mesh = tuple(int(v) for v in mesh)
    nk = int(np.prod(mesh))
    mk = tuple(int(v) for v in mk)
    if len(mk) != nk or min(mk) < nocc:
        raise ValueError("need nk band counts, each at least nocc")
    if rng is None:
        rng = np.random.Generator(np.random.PCG64(seed))
    H1 = []
    for k in range(nk):
        m = mk[k]
        c = 0.05 * _cn(rng, (m, m))
        h = 0.5 * (c + c.conj().T)
        np.fill_diagonal(h, 0.0)
        H1.append(np.diag(np.linspace(-1.0, 2.0, m)) + h)
    scale = np.exp(-np.arange(nchol) / 6.0) / np.sqrt(max(mk))
    L = [[None] * nk for _ in range(nk)]
    for Q in range(nk):
        for k in range(nk):
            if L[Q][k] is not None:
                continue
            pQ, pk = _partner(Q, k, mesh)  # pk = k - Q
            z = _cn(rng, (mk[k], mk[pk], nchol))
            if (pQ, pk) == (Q, k):
                L[Q][k] = 0.5 * (z + z.conj().transpose(1, 0, 2)) * scale
            else:
                L[Q][k] = z * scale
                L[pQ][pk] = L[Q][k].conj().transpose(1, 0, 2)
    A = []
    for k in range(nk):
        q, _ = np.linalg.qr(_cn(rng, (mk[k], nocc)))
        A.append(q)
    return RaggedSystem(mesh=mesh, mk=mk, nocc=nocc, nchol=nchol, dt=dt, H1=H1, L=L, A=A,
                        seed=seed), rng


def make_ragged_walkers(rs: RaggedSystem, nwalk: int, rng: np.random.Generator):
    """Dense walkers U[w] of shape (sum mk, nk*nocc): QR of a CN(0,1) matrix."""
    M, n = sum(rs.mk), rs.nk * rs.nocc
    U = np.empty((nwalk, M, n), dtype=np.complex128)
    for w in range(nwalk):
        q, _ = np.linalg.qr(_cn(rng, (M, n)))
        U[w] = q
    return U


def pack_ragged(rs: RaggedSystem, U=None):
    """The packed layouts of the band-padding entry: L blocks (Q-major, then k) of
    (mk[k], mk[k-Q], nchol), H1 blocks (mk[k], mk[k]), A blocks (mk[k], nocc), each flat
    and concatenated; U as given ([nwalk][sum mk][nk*nocc])."""
    nk = rs.nk
    Lr = np.concatenate([rs.L[Q][k].reshape(-1) for Q in range(nk) for k in range(nk)])
    Hr = np.concatenate([h.reshape(-1) for h in rs.H1])
    Ar = np.concatenate([a.reshape(-1) for a in rs.A])
    return Lr, Hr, Ar, (None if U is None else np.ascontiguousarray(U))
