"""Non-uniform band counts on the GPU: the padding entries against the oracle's padding (bit
for bit), and the padded system's Green's function, energy and step against the supercell
route of the ragged system."""

import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    import paper_2003_09468_amd as lib
    from synth import make_ragged_system, make_ragged_walkers, pack_ragged
    from oracle import bands as bd
    from oracle import kpoint as kp
    from oracle import supercell as sc
    from tests.gpu_cases import host, rel, phase_err

# (mesh, mk, nocc, nchol, nwalk, pad): self-paired and paired Q, m past 32, extra padding
RAGGED = {
    "line2": ((2, 1, 1), (4, 6), 2, 7, 3, 0),
    "aniso": ((2, 3, 1), (4, 5, 3, 4, 6, 5), 2, 9, 4, 2),
    "c8": ((2, 2, 2), (8, 6, 7, 8, 5, 8, 6, 7), 3, 20, 5, 0),
    "m40": ((1, 1, 2), (33, 40), 4, 11, 3, 0),
}
CASESEL = list(RAGGED) if gpu_available() else []


@pytest.mark.skipif(not gpu_available(), reason="needs a GPU")
@pytest.mark.parametrize("case", CASESEL)
def test_padded_bands_against_supercell(case):
    mesh, mk, nocc, C, W, extra = RAGGED[case]
    rs, rng = make_ragged_system(mesh, mk, nocc, C, seed=2)
    Ur = make_ragged_walkers(rs, W, rng)
    x = rng.standard_normal((1, W, rs.nk, C, 2))
    m = max(mk) + extra
    Lr, Hr, Ar, Ur_ = pack_ragged(rs, Ur)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a))  # noqa: E731
    L, H1, A, U = lib.pad_bands(mesh, mk, m, nocc, C, t(Lr), t(Hr), t(Ar), t(Ur_))
    torch.cuda.synchronize()
    Lo, Ho, Ao = bd.pad(rs, m)
    assert np.array_equal(host(L), Lo) and np.array_equal(host(H1), Ho)
    assert np.array_equal(host(A), Ao)
    assert np.array_equal(host(U), bd.pad_walkers(Ur, mk, m))
    p = lib.KptProblem(mesh, m, nocc, C, W, rs.dt, L, A)
    p.prepare(H1)
    p.set_walkers(U)
    p.greens()
    E = host(p.energy())
    Ur2, Gr = lib.unpad_bands(p, mk, U=p.U, Gh=p.Gh)
    torch.cuda.synchronize()
    assert np.array_equal(host(Ur2), Ur)
    LL, h, Af = bd.supercell(rs)
    v = sc.eri(LL)
    V0 = sc.v0_full(LL)
    ld0 = np.empty(W, dtype=complex)
    for w in range(W):
        assert rel(host(Gr)[w], sc.half_greens_full(Ur[w], Af)) < 1e-12
        ref = sc.energy_4index(h, v, sc.greens_full(Ur[w], Af))
        assert np.abs(E[w] - ref).max() < 1e-11 * np.abs(ref).sum()
        sg, la = np.linalg.slogdet(Af.conj().T @ Ur[w])
        ld0[w] = la + 1j * np.angle(sg)
    assert phase_err(host(p.logdet), ld0) < 1e-12
    # one step: the ragged walkers by the dense supercell propagator, zero padded rows
    xbar, _ = p.step(torch.from_numpy(x[0]))
    torch.cuda.synchronize()
    xb = host(xbar)
    Us, _ = lib.unpad_bands(p, mk, U=p.U)
    Us = host(Us)
    pad_rows = np.ones(rs.nk * m, dtype=bool)
    for k in range(rs.nk):
        pad_rows[k * m:k * m + mk[k]] = False
    assert not np.any(host(p.U)[:, pad_rows])
    for w in range(W):
        G = sc.greens_full(Ur[w], Af)
        xref = sc.force_bias_full(LL, G, rs.dt).reshape(rs.nk, C, 2)
        assert rel(xb[w], xref) < 1e-12
        V = sc.hs_matrix_full(LL, x[0][w].reshape(-1, 2), xref.reshape(-1, 2), rs.dt)
        Un = sc.propagate_full(Ur[w], V, h, V0, rs.dt)
        assert rel(Us[w], Un) < 1e-11
    # log overlaps of the propagated walkers against dense determinants
    ld1 = np.empty(W, dtype=complex)
    for w in range(W):
        sg, la = np.linalg.slogdet(Af.conj().T @ Us[w])
        ld1[w] = la + 1j * np.angle(sg)
    assert phase_err(host(p.logdet), ld1) < 1e-11
